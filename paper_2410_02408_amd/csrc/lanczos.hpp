// Lanczos in the M inner product with full reorthogonalisation, and the
// extreme eigenvalues of the resulting tridiagonal.
//
// Per step j (basis v_0..v_j, M-orthonormal, u_l = M v_l kept alongside so M
// is never applied forward):
//   k_spmv<LANCZOS>        v_j, u_j normalised; w = A v_j; alpha_j = v_j^T w
//   k_gram<GRAM_FIRST>     r~ = w - alpha_j u_j - beta_{j-1} u_{j-1};
//                          partial c_l = v_l^T r~            (l <= j)
//   k_gram_reduce          c_l = sum of partials (fixed order)
//   k_gram<GRAM_SECOND>    r~ -= sum_l c_l u_l; partial c_l = v_l^T r~
//   k_gram_reduce
//   k_gram<GRAM_FINAL>     r~ -= sum_l c_l u_l   (with M = I also beta_j)
//   k_apply<LANCZOS>       z~ = M^-1 r~; beta_j = sqrt(r~^T z~)
// The Gram passes are tall-skinny products over the j+1 stored vectors and
// stream 8(j+1)N bytes each: they dominate the estimate's cost at large j.
#pragma once

#include "blocks.hpp"
#include "common.hpp"

namespace bjp {

constexpr int kGramRows = 8;      // rows per thread in the Gram kernels

enum GramPass { GRAM_FIRST = 0, GRAM_SECOND = 1, GRAM_FINAL = 2 };

struct GramArgs {
    int n, chunk;            // chunk = rows per workgroup (kWG * kGramRows)
    LanczosState *ls;
    const double *w;         // FIRST: A v_j
    const double *U, *V;     // bases, vector l at l*ld (V == U when M = I)
    size_t ld;
    double *rt;              // r~, updated in place
    const double *c;         // SECOND / FINAL: coefficients of the previous pass
    double *cpart;           // FIRST / SECOND: partial coefficients [grid][ldc]
    int ldc;
    int has_m;
    double *partials;        // FINAL with M = I: per-workgroup r~^T r~
};

// Basis vectors handled per round of the Gram loops: the loads of a round are
// issued together (clamped, in-bounds row indices; rows past the chunk are
// masked by value, not by branches), so each thread has kGramUnroll *
// kGramRows loads in flight.
#ifndef BJP_GRAM_UNROLL
#define BJP_GRAM_UNROLL 4
#endif
constexpr int kGramUnroll = BJP_GRAM_UNROLL;

// The stored basis is streamed once per pass and exceeds every cache level,
// so its loads are non-temporal, which leaves the caches to r~ and the
// coefficients (measured at 128^3, 200 steps: 253 -> 226 ms for kappa(A),
// 273 -> 247 ms for kappa(M^-1 A)).
__device__ __forceinline__ double basis_load(const double *p) { return __builtin_nontemporal_load(p); }

template <int PASS>
__global__ __launch_bounds__(kWG) void k_gram(GramArgs a) {
    LanczosState *ls = a.ls;
    if (ls->done) return;
    const int j = ls->j;
    const int tid = threadIdx.x;
    const int c = xcd_chunk(blockIdx.x, gridDim.x);
    const int r0 = c * a.chunk;
    const int r1 = min(r0 + a.chunk, a.n);
    constexpr int Q = kGramRows, UN = kGramUnroll;
    double rv[Q];
    int rc[Q];
    bool ok[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int row = r0 + q * kWG + tid;
        ok[q] = row < r1;
        rc[q] = min(row, a.n - 1);
        double v = 0.0;
        if (PASS == GRAM_FIRST) {
            v = a.w[rc[q]] - ls->alpha_j * a.U[(size_t)j * a.ld + rc[q]];
            if (j > 0) v -= ls->beta_prev * a.U[(size_t)(j - 1) * a.ld + rc[q]];
        } else {
            v = a.rt[rc[q]];
        }
        rv[q] = ok[q] ? v : 0.0;
    }
    if (PASS != GRAM_FIRST) {
        // r~ -= sum_l c_l u_l, l in order
        int l = 0;
        for (; l + UN <= j + 1; l += UN) {
            double u[UN][Q];
#pragma unroll
            for (int t = 0; t < UN; ++t)
#pragma unroll
                for (int q = 0; q < Q; ++q) u[t][q] = basis_load(a.U + (size_t)(l + t) * a.ld + rc[q]);
#pragma unroll
            for (int t = 0; t < UN; ++t) {
                const double cl = a.c[l + t];
#pragma unroll
                for (int q = 0; q < Q; ++q) rv[q] = ok[q] ? rv[q] - cl * u[t][q] : 0.0;
            }
        }
        for (; l <= j; ++l) {
            const double cl = a.c[l];
            const double *ul = a.U + (size_t)l * a.ld;
#pragma unroll
            for (int q = 0; q < Q; ++q) rv[q] = ok[q] ? rv[q] - cl * basis_load(ul + rc[q]) : 0.0;
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
        if (ok[q]) a.rt[rc[q]] = rv[q];

    if (PASS != GRAM_FINAL) {
        // partial c_l = v_l^T r~ over this workgroup's rows, l in rounds of UN
        __shared__ double red[UN][kWaves];
        const int lane = tid & 63, wave = tid >> 6;
        for (int l0 = 0; l0 <= j; l0 += UN) {
            double v[UN][Q];
#pragma unroll
            for (int t = 0; t < UN; ++t) {
                const int l = min(l0 + t, j);
#pragma unroll
                for (int q = 0; q < Q; ++q) v[t][q] = basis_load(a.V + (size_t)l * a.ld + rc[q]);
            }
            double sv[UN];
#pragma unroll
            for (int t = 0; t < UN; ++t) {
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < Q; ++q) s += v[t][q] * rv[q];
                sv[t] = wave_sum(s);
            }
            if (lane == 0) {
#pragma unroll
                for (int t = 0; t < UN; ++t) red[t][wave] = sv[t];
            }
            __syncthreads();
            if (tid < UN && l0 + tid <= j) {
                double s = 0.0;
                for (int w = 0; w < kWaves; ++w) s += red[tid][w];
                a.cpart[(size_t)blockIdx.x * a.ldc + l0 + tid] = s;
            }
            __syncthreads();
        }
    } else if (!a.has_m) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) s += rv[q] * rv[q];
        const double v[1] = {s};
        block_partial<1>(v, a.partials);
    }
}

// c_l = sum over workgroups of cpart[w][l]; one workgroup per l.
__global__ __launch_bounds__(kWG) void k_gram_reduce(LanczosState *ls, const double *cpart, int ldc,
                                                     int nparts, double *c) {
    if (ls->done) return;
    const int l = blockIdx.x;
    if (l > ls->j) return;
    double s = 0.0;
    for (int w = threadIdx.x; w < nparts; w += kWG) s += cpart[(size_t)w * ldc + l];
    __shared__ double red[kWaves];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kWaves; ++w) t += red[w];
        c[l] = t;
    }
}

// Number of eigenvalues of T = tridiag(beta; alpha; beta) below x: negative
// pivots of the LDL^T factorisation of T - x I (pivots below pivmin in size
// are pushed to -pivmin).  b2[i] = beta_i^2.
__device__ __forceinline__ int sturm_count(const double *al, const double *b2, int s, double x, double pivmin) {
    double d = al[0] - x;
    if (fabs(d) < pivmin) d = -pivmin;
    int cnt = d < 0.0 ? 1 : 0;
    for (int i = 1; i < s; ++i) {
        d = al[i] - x - b2[i - 1] / d;
        if (fabs(d) < pivmin) d = -pivmin;
        cnt += d < 0.0 ? 1 : 0;
    }
    return cnt;
}

__device__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Extreme eigenvalues of the s x s Lanczos tridiagonal by Sturm-count
// multisection.  Waves 0-3 bracket the smallest eigenvalue, waves 4-7 the
// largest, at the same time.  Each round the 256 lanes of a group probe 256
// interior points of its bracket (one each: a probe's recurrence is a chain
// of divisions, so more probes per lane would only queue behind it), which
// shrinks the bracket 257-fold; the waves of a group exchange their first
// hits through LDS.  Every wave takes every round's barrier, a converged
// group included, until both groups have converged.  alpha and beta^2 are
// staged in LDS when the launch gives room (lds_steps >= s, 16 bytes a step).
constexpr int kTriWaves = 8;
constexpr int kTriLdsSteps = 4096;   // the launch stages up to this many steps (64 KB)

__global__ __launch_bounds__(64 * kTriWaves) void k_tridiag(LanczosState *ls, const double *al_g, const double *be_g,
                                                            int lds_steps) {
    constexpr int GW = kTriWaves / 2;   // waves per group
    constexpr int NP = 64 * GW;         // probes per group and round
    extern __shared__ double tl[];      // alpha [lds_steps], then beta^2 [lds_steps]
    __shared__ int firsts[2][2][GW];    // [round parity][group][wave]: first hit, NP none, -1 converged
    __shared__ double res[2];
    const int s = ls->steps_done;
    if (ls->status != BJP_OK || s <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int group = wave / GW, wig = wave % GW;
    const bool staged = s <= lds_steps;
    double *b2 = tl + lds_steps;
    if (staged) {
        for (int i = tid; i < s; i += 64 * kTriWaves) {
            tl[i] = al_g[i];
            if (i + 1 < s) b2[i] = be_g[i] * be_g[i];
        }
    }
    __syncthreads();
    // Gershgorin interval (every wave forms the same one, in the same order)
    double glo = INFINITY, ghi = -INFINITY, bmax = 1.0;
    for (int i = lane; i < s; i += 64) {
        double rad = 0.0;
        if (i > 0) rad += fabs(be_g[i - 1]);
        if (i + 1 < s) {
            rad += fabs(be_g[i]);
            bmax = fmax(bmax, be_g[i] * be_g[i]);
        }
        glo = fmin(glo, al_g[i] - rad);
        ghi = fmax(ghi, al_g[i] + rad);
    }
    glo = wave_min(glo);
    ghi = wave_max(ghi);
    bmax = wave_max(bmax);
    const double eps = 2.220446049250313e-16;
    const double pivmin = 2.2250738585072014e-308 * bmax;
    const double widen = 4.0 * eps * (fabs(glo) + fabs(ghi) + (ghi - glo)) * s + 2.0 * pivmin;
    const int target = group == 0 ? 1 : s;
    double lo = glo - widen, hi = ghi + widen;
    for (int round = 0; round < 64; ++round) {
        const int par = round & 1;
        const bool conv = hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) || hi - lo <= pivmin;
        const double h = (hi - lo) / (NP + 1.0);
        if (!conv) {
            const double x = lo + h * (wig * 64 + lane + 1);
            int cnt;
            if (staged) {
                cnt = sturm_count(tl, b2, s, x, pivmin);
            } else {
                // beta^2 formed per step, the same product as the staged one
                double d = al_g[0] - x;
                if (fabs(d) < pivmin) d = -pivmin;
                cnt = d < 0.0 ? 1 : 0;
                for (int i = 1; i < s; ++i) {
                    d = al_g[i] - x - (be_g[i - 1] * be_g[i - 1]) / d;
                    if (fabs(d) < pivmin) d = -pivmin;
                    cnt += d < 0.0 ? 1 : 0;
                }
            }
            const unsigned long long hit = __ballot(cnt >= target);
            if (lane == 0) firsts[par][group][wig] = hit ? wig * 64 + __ffsll((long long)hit) - 1 : NP;
        } else if (lane == 0) {
            firsts[par][group][wig] = -1;
        }
        __syncthreads();
        if (firsts[par][0][0] < 0 && firsts[par][1][0] < 0) break;   // the same for every thread
        if (!conv) {
            // the first probe (in order) that reached the target count
            int first = NP;
#pragma unroll
            for (int w = 0; w < GW; ++w) first = min(first, firsts[par][group][w]);
            const double nlo = first == 0 ? lo : lo + h * first;
            const double nhi = first == NP ? hi : lo + h * (first + 1);
            lo = nlo;
            hi = nhi;
        }
    }
    if (wig == 0 && lane == 0) res[group] = 0.5 * (lo + hi);
    __syncthreads();
    if (tid == 0) {
        ls->theta_min = res[0];
        ls->theta_max = res[1];
        ls->kappa = res[1] / res[0];
    }
}

}  // namespace bjp
