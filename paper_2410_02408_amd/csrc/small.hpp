// PCG for a small system in one workgroup.
//
// At a few thousand rows every kernel of the multi-launch solver is a few
// microseconds of fixed cost (launch, prologue, a handful of loads), so an
// iteration costs three launch latencies whatever its bytes.  Here one
// workgroup of kSmallWG threads runs the whole solve: the same algorithm,
// scalar decisions (finish_decide) and stopping rule, true-residual check and
// residual replacement as bjp_pcg_solve, with workgroup barriers between the
// phases instead of kernel boundaries.  Thread t owns rows t, t + kSmallWG,
// ...: it forms their products row by row (entries in storage order), their
// x, r and p updates; the block-inverse application runs packet by packet on
// the waves (wave w takes packets w, w + kSmallWaves, ...).  Every total is a
// fixed-order workgroup reduction, so the solve is deterministic.  The
// vectors live in the solver's workspace and stay in the caches.
#pragma once

#include "blocks.hpp"
#include "common.hpp"
#include "finish.hpp"

namespace bjp {

constexpr int kSmallWG = 512;
constexpr int kSmallWaves = kSmallWG / 64;
constexpr int kSmallMaxRows = 8 * kSmallWG;   // at most 8 rows per thread
constexpr int kSmallMaxMeanRow = 32;          // longer rows take the multi-launch products

struct SmallArgs {
    int n;
    const int32_t *rp, *ci;
    const double *val;
    const double *b;
    double *x;
    double *r, *z, *p, *q;   // z == r without a preconditioner
    // the preconditioner (unused without one)
    int nblocks, num_packets, uniform_nb;
    const int32_t *off;
    const void *tiles;
    double tol;
    int max_iter, max_repl, x0_given;
    double *hist;            // optional residual history
    PcgState *out;           // the final state
    int32_t *repl_out;       // replacements made
};

// Totals of NQ per-thread values over the workgroup, in a fixed order; every
// thread receives them.  Ends with a barrier, so `red` can be reused and every
// store made before the call is visible to the whole workgroup after it.
template <int NQ>
__device__ __forceinline__ void small_sum(double (&v)[NQ], double (*red)[kSmallWaves]) {
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
        for (int w = 0; w < kSmallWaves; ++w) t += red[q][w];
        v[q] = t;
    }
    __syncthreads();
}

// (A u)_i, entries in storage order.
__device__ __forceinline__ double small_row(const SmallArgs &a, int i, const double *u) {
    double s = 0.0;
    const int k1 = a.rp[i + 1];
    for (int k = a.rp[i]; k < k1; ++k) s += a.val[k] * u[a.ci[k]];
    return s;
}

// z = M^-1 r over every packet; this thread's share of r^T z and r^T r.
template <int G, typename TS>
__device__ __forceinline__ void small_apply(const SmallArgs &a, double &rz, double &rr) {
    constexpr int P = 64 / G, E = packet_elems(G);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane / G, i = lane % G;
    const TS *tiles = static_cast<const TS *>(a.tiles);
    for (int pk = wave; pk < a.num_packets; pk += kSmallWaves) {
        const int t = pk * P + g;
        int s, nn;
        if (a.uniform_nb > 0) {
            s = t * a.uniform_nb;
            nn = max(0, min(a.uniform_nb, a.n - s));
        } else {
            const int tc = min(t, a.nblocks - 1);
            s = t < a.nblocks ? a.off[tc] : 0;
            nn = t < a.nblocks ? a.off[tc + 1] - a.off[tc] : 0;
        }
        const bool act = i < nn;
        const int rc = min(s + i, a.n - 1);
        const double rv = act ? a.r[rc] : 0.0;
        TS dv[G / 2 + 1];
        packet_load<G, TS>(tiles + (size_t)pk * E, lane, g, i, dv);
        const TS zv = packet_product<G, TS>(dv, g, i, nn, (TS)rv);
        if (act) {
            const double z = (double)zv;
            a.z[s + i] = z;
            rz += rv * z;
            rr += rv * rv;
        }
    }
}

template <int G, typename TS, bool HAS_M>
__global__ __launch_bounds__(kSmallWG) void k_pcg_small(SmallArgs a) {
    __shared__ double red[2][kSmallWaves];
    const int tid = threadIdx.x, n = a.n;
    PcgState L;
    L.rho = L.alpha = L.beta = L.bnorm2 = 0.0;
    L.tol = a.tol;
    L.relres = L.relres_true = 0.0;
    L.it = 0;
    L.done = 0;
    L.status = BJP_OK;
    L.max_iter = a.max_iter;
    L.zero_rhs = 0;
    L.pending = L.xpend = L.pad = 0;
    FinishArgs f{};
    f.hist = tid == 0 ? a.hist : nullptr;   // one thread records the history

    // r = b - A x0 (x0 = 0 unless given), ||b||^2, ||r||^2
    {
        double v[2] = {0.0, 0.0};
        for (int i = tid; i < n; i += kSmallWG) {
            const double bi = a.b[i];
            double ri = bi;
            if (a.x0_given) ri = bi - small_row(a, i, a.x);
            else a.x[i] = 0.0;
            a.r[i] = ri;
            v[0] += bi * bi;
            v[1] += ri * ri;
        }
        small_sum<2>(v, red);
        finish_decide<FIN_RESID_START>(f, &L, nullptr, v);
    }
    int repl = 0;
    for (;;) {
        if (!L.done) {
            // (re)start the direction from r: z = M^-1 r, rho = r^T z, p = z
            double v[1] = {0.0};
            if constexpr (HAS_M) {
                double rr = 0.0;
                small_apply<G, TS>(a, v[0], rr);
            } else {
                for (int i = tid; i < n; i += kSmallWG) v[0] += a.r[i] * a.r[i];
            }
            small_sum<1>(v, red);
            finish_decide<FIN_PCG_START>(f, &L, nullptr, v);
            if (!L.done)
                for (int i = tid; i < n; i += kSmallWG) a.p[i] = a.z[i];
        }
        while (!L.done) {
            __syncthreads();   // p complete before it is gathered
            double sg[1] = {0.0};
            for (int i = tid; i < n; i += kSmallWG) {
                const double qi = small_row(a, i, a.p);
                a.q[i] = qi;
                sg[0] += a.p[i] * qi;
            }
            small_sum<1>(sg, red);
            finish_decide<FIN_SIGMA>(f, &L, nullptr, sg);
            if (L.done) break;
            const double alpha = L.alpha;
            for (int i = tid; i < n; i += kSmallWG) {
                a.x[i] = __builtin_fma(alpha, a.p[i], a.x[i]);
                a.r[i] = __builtin_fma(-alpha, a.q[i], a.r[i]);
            }
            if constexpr (HAS_M) {
                double u[2] = {0.0, 0.0};
                __syncthreads();   // r complete before the packets read it
                small_apply<G, TS>(a, u[0], u[1]);
                small_sum<2>(u, red);
                finish_decide<FIN_PCG_UPDATE>(f, &L, nullptr, u);
            } else {
                double u[1] = {0.0};
                for (int i = tid; i < n; i += kSmallWG) u[0] += a.r[i] * a.r[i];
                small_sum<1>(u, red);
                finish_decide<FIN_PCG_UPDATE_I>(f, &L, nullptr, u);
            }
            if (!L.done) {
                const double beta = L.beta;
                for (int i = tid; i < n; i += kSmallWG) a.p[i] = __builtin_fma(beta, a.p[i], a.z[i]);
            }
        }
        if (L.zero_rhs) {
            for (int i = tid; i < n; i += kSmallWG) a.x[i] = 0.0;
            L.relres_true = 0.0;
            break;
        }
        // the true residual r = b - A x (also the residual a replacement restarts from)
        __syncthreads();   // x complete before it is gathered
        {
            double v[2] = {0.0, 0.0};
            for (int i = tid; i < n; i += kSmallWG) {
                const double bi = a.b[i];
                const double ri = bi - small_row(a, i, a.x);
                a.r[i] = ri;
                v[0] += bi * bi;
                v[1] += ri * ri;
            }
            small_sum<2>(v, red);
            finish_decide<FIN_RESID_TRUE>(f, &L, nullptr, v);
        }
        if (L.status != BJP_OK || L.relres_true <= L.tol) break;
        // a replacement needs an iteration to follow it
        if (repl >= a.max_repl || L.it >= L.max_iter) {
            L.status = BJP_ENOCONV;
            break;
        }
        ++repl;
        L.done = 0;
    }
    if (tid == 0) {
        store_state(a.out, L);
        *a.repl_out = repl;
    }
}

}  // namespace bjp
