// PCG for a small system in one workgroup.
//
// At a few thousand rows every kernel of the multi-launch solver is a few
// microseconds of fixed cost (launch, prologue, a handful of loads), so an
// iteration costs three launch latencies whatever its bytes.  Here one
// workgroup of kSmallWG threads runs the whole solve: the same algorithm,
// scalar decisions (finish_decide) and stopping rule, true-residual check and
// residual replacement as bjp_pcg_solve, with workgroup barriers between the
// phases instead of kernel boundaries.  Thread t owns rows t, t + kSmallWG,
// ...: it keeps their x, r, p, z and q in registers, forms their products row
// by row (entries in storage order) gathering from the direction held in LDS;
// the block-inverse application runs packet by packet on the waves (wave w
// takes packets w, w + kSmallWaves, ...), in registers when the blocks are
// uniform and as wide as their lane group (a packet's rows are then its
// lanes' own rows), else on r staged in LDS.  Every total is a fixed-order
// workgroup reduction, so the solve is deterministic.  Only the
// matrix and the block inverses are read in an iteration; whatever of them
// fits in LDS beside the vectors (the inverse packets first, then the CSR
// values and columns; 160 KB per workgroup on gfx950) is copied there once
// per solve, which takes their L2 round trips off every iteration.
#pragma once

#include <type_traits>

#include "blocks.hpp"
#include "common.hpp"
#include "finish.hpp"

namespace bjp {

constexpr int kSmallWG = 512;
constexpr int kSmallWaves = kSmallWG / 64;
constexpr int kSmallMaxRows = 4 * kSmallWG;   // at most 4 rows per thread
constexpr int kSmallMaxMeanRow = 32;          // longer rows take the multi-launch products
// dynamic LDS a one-workgroup kernel may take (gfx950: 160 KB per workgroup,
// less what the kernels declare statically)
constexpr size_t kSmallLdsBytes = 160 * 1024 - 2048;
// what a one-workgroup kernel keeps in LDS besides its vectors (bits)
constexpr int kResTiles = 1, kResCsr = 2;

struct SmallArgs {
    int n, nnz;
    int tiles_bytes;         // bytes of the inverse packets (copied to LDS with kResTiles)
    const int32_t *rp, *ci;
    const double *val;
    const double *b;
    double *x;
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
// thread receives them.  One barrier: every store made before the call is
// visible to the whole workgroup after it.  `red` is read after that barrier,
// so it must not be written again before every thread has passed another
// barrier (callers alternate two buffers, or put a barrier between).
template <int NQ, int WAVES = kSmallWaves>
__device__ __forceinline__ void small_sum(double (&v)[NQ], double (*red)[WAVES]) {
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
        for (int w = 0; w < WAVES; ++w) t += red[q][w];
        v[q] = t;
    }
}

// This thread's rows: row(u) = threadIdx.x + u * kSmallWG, u < kSmallR.
constexpr int kSmallR = kSmallMaxRows / kSmallWG;

// z = M^-1 r over every packet, in place in w (r in, z out; each row is read
// and written by the one lane that owns it in its packet); this thread's
// share of r^T z and r^T r.
template <int G, typename TS, int WAVES = kSmallWaves>
__device__ __forceinline__ void small_apply(int n, int nblocks, int num_packets, int uniform_nb,
                                            const int32_t *off, const void *tiles_, double *w, double &rz,
                                            double &rr) {
    constexpr int P = 64 / G, E = packet_elems(G);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane / G, i = lane % G;
    const TS *tiles = static_cast<const TS *>(tiles_);
    for (int pk = wave; pk < num_packets; pk += WAVES) {
        const int t = pk * P + g;
        int s, nn;
        if (uniform_nb > 0) {
            s = t * uniform_nb;
            nn = max(0, min(uniform_nb, n - s));
        } else {
            const int tc = min(t, nblocks - 1);
            s = t < nblocks ? off[tc] : 0;
            nn = t < nblocks ? off[tc + 1] - off[tc] : 0;
        }
        const bool act = i < nn;
        const int rc = min(s + i, n - 1);
        TS dv[G / 2 + 1];
        packet_load<G, TS>(tiles + (size_t)pk * E, lane, g, i, dv);
        const double rv = act ? w[rc] : 0.0;
        const TS zv = packet_product<G, TS>(dv, g, i, nn, (TS)rv);
        if (act) {
            const double z = (double)zv;
            w[s + i] = z;
            rz += rv * z;
            rr += rv * rv;
        }
    }
}

// z = M^-1 r for this thread's rows, in registers, when the blocks are
// uniform of G rows (G = the group width): packet pk then holds rows 64 pk ..
// 64 pk + 63, lane l row 64 pk + l, so wave w's packets w, w + kSmallWaves,
// ... hold exactly the rows of its threads (row(k) = tid + k kSmallWG), and
// no value crosses a thread.  The same operations in the same order as
// small_apply, so the same results.
template <int G, typename TS>
__device__ __forceinline__ void small_apply_regs(int n, int num_packets, const void *tiles_,
                                                 const double (&r)[kSmallR], double (&z)[kSmallR], double &rz,
                                                 double &rr) {
    constexpr int P = 64 / G, E = packet_elems(G);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane / G, i = lane % G;
    const TS *tiles = static_cast<const TS *>(tiles_);
#pragma unroll
    for (int k = 0; k < kSmallR; ++k) {
        const int pk = wave + k * kSmallWaves;   // the same for the whole wave
        z[k] = 0.0;
        if (pk < num_packets) {
            const int s = (pk * P + g) * G;
            const int nn = max(0, min(G, n - s));
            const bool act = i < nn;
            TS dv[G / 2 + 1];
            packet_load<G, TS>(tiles + (size_t)pk * E, lane, g, i, dv);
            const TS zv = packet_product<G, TS>(dv, g, i, nn, (TS)(act ? r[k] : 0.0));
            if (act) {
                z[k] = (double)zv;
                rz += r[k] * z[k];
                rr += r[k] * r[k];
            }
        }
    }
}

// The vectors live in LDS and registers: u (the vector the products gather:
// p, or x for a residual) and w (r staged for an application whose blocks
// cross threads, z after it), n doubles each; every thread keeps x, r, p, z
// and q = A p of its own rows in registers and the extents of its rows' CSR
// entries.
// Copies what RES names to LDS at `rest` (16-byte aligned, after the
// kernel's vectors); the pointers then refer to the copies.  Ends with a
// barrier.
template <int RES>
__device__ __forceinline__ void small_stage(char *rest, int nnz, int tiles_bytes, const void *&tiles,
                                            const double *&val, const int32_t *&ci) {
    if constexpr ((RES & kResTiles) != 0) {
        const uint4 *src = static_cast<const uint4 *>(tiles);
        uint4 *dst = reinterpret_cast<uint4 *>(rest);
        for (int q = threadIdx.x; q < tiles_bytes / 16; q += kSmallWG) dst[q] = src[q];
        tiles = rest;
        rest += tiles_bytes;
    }
    if constexpr ((RES & kResCsr) != 0) {
        double *lv = reinterpret_cast<double *>(rest);
        int32_t *lc = reinterpret_cast<int32_t *>(lv + nnz);
        for (int e = threadIdx.x; e < nnz; e += kSmallWG) {
            lv[e] = val[e];
            lc[e] = ci[e];
        }
        val = lv;
        ci = lc;
    }
    __syncthreads();
}

// LDS bytes of what RES names (the vectors not included)
__host__ __device__ constexpr size_t small_stage_bytes(int res, int nnz, int tiles_bytes) {
    return ((res & kResTiles) ? (size_t)tiles_bytes : 0) + ((res & kResCsr) ? (size_t)nnz * 12 : 0);
}

template <int G, typename TS, bool HAS_M, int RES>
__global__ __launch_bounds__(kSmallWG) void k_pcg_small(SmallArgs a) {
    extern __shared__ double lds[];
    double *u = lds, *w = lds + a.n;
    __shared__ double red[2][2][kSmallWaves];   // two buffers, used in turn
    const int tid = threadIdx.x, n = a.n;
    int rb = 0;
    auto sum = [&](auto &v) {
        small_sum(v, red[rb]);
        rb ^= 1;
    };
    // uniform blocks as wide as the group: the application stays in registers
    // (groups of up to 16 lanes; wider packets leave too few registers)
    const bool aligned = HAS_M && G <= 16 && a.uniform_nb == G;
    const void *tiles = a.tiles;
    const double *val = a.val;
    const int32_t *ci = a.ci;
    small_stage<RES>(reinterpret_cast<char *>(lds + 2 * (size_t)n), a.nnz, a.tiles_bytes, tiles, val, ci);
    int kb[kSmallR], ke[kSmallR];
    double x[kSmallR], r[kSmallR], p[kSmallR], z[kSmallR];
#pragma unroll
    for (int k = 0; k < kSmallR; ++k) {
        const int i = tid + k * kSmallWG;
        kb[k] = i < n ? a.rp[i] : 0;
        ke[k] = i < n ? a.rp[i + 1] : 0;
        x[k] = r[k] = p[k] = z[k] = 0.0;
    }
    // (A u) of this thread's row k, entries in storage order
    auto row = [&](int k) {
        double acc = 0.0;
        for (int e = kb[k]; e < ke[k]; ++e) acc += val[e] * u[ci[e]];
        return acc;
    };
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
#pragma unroll
        for (int k = 0; k < kSmallR; ++k) {
            const int i = tid + k * kSmallWG;
            if (i < n) {
                x[k] = a.x0_given ? a.x[i] : 0.0;
                u[i] = x[k];
            }
        }
        __syncthreads();
        double v[2] = {0.0, 0.0};
#pragma unroll
        for (int k = 0; k < kSmallR; ++k) {
            const int i = tid + k * kSmallWG;
            if (i < n) {
                const double bi = a.b[i];
                r[k] = a.x0_given ? bi - row(k) : bi;
                v[0] += bi * bi;
                v[1] += r[k] * r[k];
            }
        }
        sum(v);
        finish_decide<FIN_RESID_START>(f, &L, nullptr, v);
    }
    // z = M^-1 r (in registers, or in w until fetch_z after the next
    // barrier); this thread's share of r^T z (and r^T r)
    auto precondition = [&](double &rz, double &rr) {
        if constexpr (HAS_M) {
            if (aligned) {
                if constexpr (G <= 16) small_apply_regs<G, TS>(n, a.num_packets, tiles, r, z, rz, rr);
            } else {
#pragma unroll
                for (int k = 0; k < kSmallR; ++k) {
                    const int i = tid + k * kSmallWG;
                    if (i < n) w[i] = r[k];
                }
                __syncthreads();   // r complete before the packets read it
                small_apply<G, TS>(a.n, a.nblocks, a.num_packets, a.uniform_nb, a.off, tiles, w, rz, rr);
            }
        } else {
#pragma unroll
            for (int k = 0; k < kSmallR; ++k) {
                const int i = tid + k * kSmallWG;
                z[k] = r[k];
                if (i < n) rz += r[k] * r[k];
            }
            rr = rz;
        }
    };
    // z of this thread's rows from w (written by other lanes: after a barrier)
    auto fetch_z = [&]() {
        if (HAS_M && !aligned) {
#pragma unroll
            for (int k = 0; k < kSmallR; ++k) {
                const int i = tid + k * kSmallWG;
                z[k] = i < n ? w[i] : 0.0;
            }
        }
    };
    int repl = 0;
    for (;;) {
        if (!L.done) {
            // (re)start the direction from r: z = M^-1 r, rho = r^T z, p = z
            double v[1] = {0.0};
            double rr = 0.0;
            precondition(v[0], rr);
            sum(v);
            finish_decide<FIN_PCG_START>(f, &L, nullptr, v);
            if (!L.done) {
                fetch_z();
#pragma unroll
                for (int k = 0; k < kSmallR; ++k) {
                    const int i = tid + k * kSmallWG;
                    if (i < n) {
                        p[k] = z[k];
                        u[i] = p[k];
                    }
                }
            }
        }
        while (!L.done) {
            __syncthreads();   // p complete in u before it is gathered
            // q = A p
            double sg[1] = {0.0};
            double q[kSmallR];
#pragma unroll
            for (int k = 0; k < kSmallR; ++k) {
                const int i = tid + k * kSmallWG;
                q[k] = 0.0;
                if (i < n) {
                    q[k] = row(k);
                    sg[0] += p[k] * q[k];
                }
            }
            sum(sg);
            finish_decide<FIN_SIGMA>(f, &L, nullptr, sg);
            if (L.done) break;
            const double alpha = L.alpha;
#pragma unroll
            for (int k = 0; k < kSmallR; ++k) {
                const int i = tid + k * kSmallWG;
                if (i < n) {
                    x[k] = __builtin_fma(alpha, p[k], x[k]);
                    r[k] = __builtin_fma(-alpha, q[k], r[k]);
                }
            }
            double t[2] = {0.0, 0.0};
            precondition(t[0], t[1]);
            if constexpr (HAS_M) {
                sum(t);
                finish_decide<FIN_PCG_UPDATE>(f, &L, nullptr, t);
            } else {
                double t1[1] = {t[0]};
                sum(t1);
                finish_decide<FIN_PCG_UPDATE_I>(f, &L, nullptr, t1);
            }
            if (!L.done) {
                fetch_z();
                const double beta = L.beta;
#pragma unroll
                for (int k = 0; k < kSmallR; ++k) {
                    const int i = tid + k * kSmallWG;
                    if (i < n) {
                        p[k] = __builtin_fma(beta, p[k], z[k]);
                        u[i] = p[k];
                    }
                }
            }
        }
        if (L.zero_rhs) {
#pragma unroll
            for (int k = 0; k < kSmallR; ++k) x[k] = 0.0;
            L.relres_true = 0.0;
            break;
        }
        // the true residual r = b - A x (also the residual a replacement restarts from)
        __syncthreads();   // every gather of u is done before x replaces p there
#pragma unroll
        for (int k = 0; k < kSmallR; ++k) {
            const int i = tid + k * kSmallWG;
            if (i < n) u[i] = x[k];
        }
        __syncthreads();
        {
            double v[2] = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < kSmallR; ++k) {
                const int i = tid + k * kSmallWG;
                if (i < n) {
                    const double bi = a.b[i];
                    r[k] = bi - row(k);
                    v[0] += bi * bi;
                    v[1] += r[k] * r[k];
                }
            }
            sum(v);
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
#pragma unroll
    for (int k = 0; k < kSmallR; ++k) {
        const int i = tid + k * kSmallWG;
        if (i < n) a.x[i] = x[k];
    }
    if (tid == 0) {
        store_state(a.out, L);
        *a.repl_out = repl;
    }
}

// ---------------------------------------------------------------------------
// Lanczos with CGS2 reorthogonalisation for a small system in one workgroup:
// the steps of the multi-launch estimate (k_spmv LANCZOS, k_gram, the
// application, the FIN_LZ_* decisions) with workgroup barriers in place of
// launches.  The basis (U, V) is kept in the workspace, where it stays in the
// caches; a step streams it four times.  The two halves of a Gram pass are
// split differently:
//   coefficients c_l = v_l^T r~: a wave computes whole coefficients (wave w
//     takes l = w*CP .. w*CP+CP-1, then every kSmallWaves*CP-th group), each
//     lane holding rows lane, lane+64, ... of r~ in registers (staged once
//     per pass through LDS), so each coefficient takes one wave reduction
//     and no exchange between waves;
//   r~ -= sum_l c_l u_l: by rows, each thread its own, l in order, with the
//     loads of kLzUnroll basis vectors in flight (deeper rounds, and rounds
//     reading basis vectors cached in LDS instead of L2, measured no faster:
//     a round is bound by its own instruction and reduction latency).
// The vector the product gathers, r~ / z~ of the application and the
// coefficients are staged in LDS, and after them whatever of the inverse
// packets and the CSR fits (as in the solver); each thread's rows of r, z,
// u_j, u_{j-1} are in registers.  The scalar decisions are taken by thread 0
// on a state in LDS that every thread then reads.
// ---------------------------------------------------------------------------
constexpr int kLzUnroll = 8;                  // basis vectors per round of the update loop
constexpr int kLzDotLoads = 32;               // basis loads in flight per lane in the dot loop
constexpr int kSmallMaxSteps = 2048;          // the coefficients live in LDS
// LDS doubles for the coefficients (steps + 1, even, so what follows is
// 16-byte aligned)
__host__ __device__ constexpr int lanczos_coef_slots(int steps) { return (steps + 2) & ~1; }

// Wave totals of UN per-lane values at once (UN a power of two, at most 64).
// In each of the first log2(UN) butterfly stages a lane keeps half of its
// values and adds its partner's copies of them, handing the other half to
// the partner; the remaining stages add single values.  Lane L ends with the
// total of value L / (64 / UN).  Fixed order, so deterministic.
template <int H, int OFF>
__device__ __forceinline__ void butterfly_stage(double *s, int lane) {
    if constexpr (H >= 1) {
        const bool hi = (lane & OFF) != 0;
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const double keep = hi ? s[H + k] : s[k];
            const double give = hi ? s[k] : s[H + k];
            s[k] = keep + __shfl_xor(give, OFF, 64);
        }
        butterfly_stage<H / 2, OFF / 2>(s, lane);
    }
}
template <int UN>
__device__ __forceinline__ double wave_sums_transposed(double (&s)[UN]) {
    const int lane = threadIdx.x & 63;
    butterfly_stage<UN / 2, 32>(s, lane);
    double v = s[0];
#pragma unroll
    for (int off = 32 / UN; off >= 1; off /= 2) v += __shfl_xor(v, off, 64);
    return v;
}

struct LanczosSmallArgs {
    int n, nnz;
    int tiles_bytes;     // bytes of the inverse packets (copied to LDS with kResTiles)
    const int32_t *rp, *ci;
    const double *val;
    int nblocks, num_packets, uniform_nb;
    const int32_t *off;
    const void *tiles;
    const double *v0;
    int steps;
    double *U, *V;       // basis vector l at l * ld (V == U without a preconditioner)
    size_t ld;
    double *alpha, *beta;
    LanczosState *ls;    // the final state (read by k_tridiag and the host)
};

template <int G, typename TS, bool HAS_M, int RES>
__global__ __launch_bounds__(kSmallWG) void k_lanczos_small(LanczosSmallArgs a) {
    constexpr int WG = kSmallWG, W = kSmallWaves, R = kSmallR;
    extern __shared__ double lds[];
    const int n = a.n, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double *vg = lds, *w = lds + n, *cf = lds + 2 * n;   // gathered vector / staged r~, z~, coefficients
    __shared__ double sred[1][W];
    __shared__ LanczosState S;
    const void *tiles = a.tiles;
    const double *val = a.val;
    const int32_t *ci = a.ci;
    small_stage<RES>(reinterpret_cast<char *>(cf + lanczos_coef_slots(a.steps)), a.nnz, a.tiles_bytes, tiles, val,
                     ci);
    int kb[R], ke[R];
    double r[R], z[R], uj[R], up[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = tid + k * WG;
        kb[k] = i < n ? a.rp[i] : 0;
        ke[k] = i < n ? a.rp[i + 1] : 0;
        r[k] = i < n ? a.v0[i] : 0.0;
        z[k] = uj[k] = up[k] = 0.0;
    }
    // clamped row index of slot k (rows past n are masked by value)
    auto row_of = [&](int k) { return min(tid + k * WG, n - 1); };
    // a wave whose upper half of slots holds no row below n skips their loads
    // in the update loop (a wave-uniform branch)
    const bool half_live = (R / 2) * WG + __builtin_amdgcn_readfirstlane(wave) * 64 >= n;
    // c_l = v_l^T r~ for every l <= j, r~ staged in vg; NM = 64-row chunks per
    // lane, held in registers up to 16 of them (read from LDS beyond that)
    auto gram_dots = [&](auto nm_tag, int j) {
        constexpr int NM = decltype(nm_tag)::value;
        constexpr int CP = kLzDotLoads / NM > 1 ? kLzDotLoads / NM : 1;   // coefficients per round
        constexpr bool IN_REGS = NM <= 16;
        double rg[IN_REGS ? NM : 1];
        auto rt = [&](int m) {
            const int i = lane + 64 * m;
            return i < n ? vg[i] : 0.0;
        };
        if constexpr (IN_REGS) {
#pragma unroll
            for (int m = 0; m < NM; ++m) rg[m] = rt(m);
        }
        // rows in halves of at most 16 chunks per lane when r~ is read from LDS
        constexpr int MH = IN_REGS ? NM : 16;
        for (int l0 = wave * CP; l0 <= j; l0 += W * CP) {
            double sv[CP];
#pragma unroll
            for (int c = 0; c < CP; ++c) sv[c] = 0.0;
#pragma unroll 1
            for (int m0 = 0; m0 < NM; m0 += MH) {
                double bv[CP][MH];
#pragma unroll
                for (int c = 0; c < CP; ++c) {
                    const double *vl = a.V + (size_t)min(l0 + c, j) * a.ld;
#pragma unroll
                    for (int m = 0; m < MH; ++m) bv[c][m] = vl[min(lane + 64 * (m0 + m), n - 1)];
                }
#pragma unroll
                for (int c = 0; c < CP; ++c)
#pragma unroll
                    for (int m = 0; m < MH; ++m)
                        sv[c] += bv[c][m] * (IN_REGS ? rg[IN_REGS ? m : 0] : rt(m0 + m));
            }
            const double tot = wave_sums_transposed<CP>(sv);
            const int c = lane / (64 / CP);
            if ((lane & (64 / CP - 1)) == 0 && l0 + c <= j) cf[l0 + c] = tot;
        }
    };
    // r~ -= sum_{l <= j} c_l u_l over this thread's rows, l in order
    auto gram_axpy = [&](auto rl_tag, int j) {
        constexpr int RL = decltype(rl_tag)::value;
        constexpr int UN = kLzUnroll;
        int l = 0;
        for (; l + UN <= j + 1; l += UN) {
            double bu[UN][RL];
#pragma unroll
            for (int t = 0; t < UN; ++t) {
                const double *ul = a.U + (size_t)(l + t) * a.ld;
#pragma unroll
                for (int k = 0; k < RL; ++k) bu[t][k] = ul[row_of(k)];
            }
#pragma unroll
            for (int t = 0; t < UN; ++t) {
                const double cl = cf[l + t];
#pragma unroll
                for (int k = 0; k < RL; ++k) r[k] -= cl * bu[t][k];
            }
        }
        for (; l <= j; ++l) {
            const double cl = cf[l];
            const double *ul = a.U + (size_t)l * a.ld;
#pragma unroll
            for (int k = 0; k < RL; ++k) r[k] -= cl * ul[row_of(k)];
        }
    };
    if (tid == 0) {
        S.invb = S.beta_prev = S.alpha_j = S.scale = 0.0;
        S.theta_min = S.theta_max = S.kappa = 0.0;
        S.j = 0;
        S.done = 0;
        S.status = BJP_OK;
        S.steps_done = 0;
        S.steps = a.steps;
        S.pad = 0;
    }
    FinishArgs f{};
    f.alpha_out = a.alpha;
    f.beta_out = a.beta;
    // z = M^-1 r (own rows, through w); returns this thread's share of r^T z
    auto precondition = [&]() -> double {
        double rz = 0.0;
        if constexpr (HAS_M) {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int i = tid + k * WG;
                if (i < n) w[i] = r[k];
            }
            __syncthreads();
            double rr = 0.0;
            small_apply<G, TS>(a.n, a.nblocks, a.num_packets, a.uniform_nb, a.off, tiles, w, rz, rr);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int i = tid + k * WG;
                z[k] = i < n ? w[i] : 0.0;
            }
        } else {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                z[k] = r[k];
                rz += r[k] * r[k];
            }
        }
        return rz;
    };
    // thread 0 takes decision OP on the totals; every thread then reads S
    auto decide = [&](auto op_tag, double (&v)[1]) {
        constexpr int OP = decltype(op_tag)::value;
        small_sum<1>(v, sred);
        if (tid == 0) finish_decide<OP>(f, nullptr, &S, v);
        __syncthreads();
    };
    {
        double v[1] = {precondition()};
        decide(std::integral_constant<int, FIN_LZ_START>{}, v);
    }
    while (!S.done) {
        const int j = S.j;
        const double invb = S.invb;
        // v_j = z~ / beta, u_j = r~ / beta: stored, and v_j staged for the product
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int i = tid + k * WG;
            up[k] = uj[k];
            uj[k] = r[k] * invb;
            if (i < n) {
                const double vj = z[k] * invb;
                a.V[(size_t)j * a.ld + i] = vj;
                if (HAS_M) a.U[(size_t)j * a.ld + i] = uj[k];
                vg[i] = vj;
            }
        }
        __syncthreads();
        // w = A v_j, alpha_j = v_j^T w; r~ = w - alpha_j u_j - beta_{j-1} u_{j-1}
        {
            double v[1] = {0.0};
#pragma unroll
            for (int k = 0; k < R; ++k) {
                if (tid + k * WG < n) {
                    double acc = 0.0;
                    for (int e = kb[k]; e < ke[k]; ++e) acc += val[e] * vg[ci[e]];
                    r[k] = acc;   // w, turned into r~ below
                    v[0] += vg[tid + k * WG] * acc;
                }
            }
            decide(std::integral_constant<int, FIN_LZ_ALPHA>{}, v);
        }
        if (S.done) break;
        const double al = S.alpha_j, bp = S.beta_prev;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            r[k] -= al * uj[k];
            if (j > 0) r[k] -= bp * up[k];
        }
        // classical Gram-Schmidt, twice: c_l = v_l^T r~ (l <= j), r~ -= sum_l c_l u_l
        for (int pass = 0; pass < 2; ++pass) {
            // r~ staged in vg (free since the product); every gather of v_j
            // is done, as a decision's barrier has passed since
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int i = tid + k * WG;
                if (i < n) vg[i] = r[k];
            }
            __syncthreads();
            if (n <= 256)
                gram_dots(std::integral_constant<int, 4>{}, j);
            else if (n <= 512)
                gram_dots(std::integral_constant<int, 8>{}, j);
            else if (n <= 1024)
                gram_dots(std::integral_constant<int, 16>{}, j);
            else
                gram_dots(std::integral_constant<int, 32>{}, j);
            __syncthreads();   // cf complete; vg read by every wave
            if (half_live)
                gram_axpy(std::integral_constant<int, R / 2>{}, j);
            else
                gram_axpy(std::integral_constant<int, R>{}, j);
        }
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (tid + k * WG >= n) r[k] = 0.0;
        // z~ = M^-1 r~, beta_j = sqrt(r~^T z~)
        double v[1] = {precondition()};
        decide(std::integral_constant<int, FIN_LZ_BETA>{}, v);
    }
    if (tid == 0) {
        a.ls->invb = S.invb;
        a.ls->beta_prev = S.beta_prev;
        a.ls->alpha_j = S.alpha_j;
        a.ls->scale = S.scale;
        a.ls->theta_min = S.theta_min;
        a.ls->theta_max = S.theta_max;
        a.ls->kappa = S.kappa;
        a.ls->j = S.j;
        a.ls->done = S.done;
        a.ls->status = S.status;
        a.ls->steps_done = S.steps_done;
        a.ls->steps = S.steps;
        a.ls->pad = 0;
    }
}

}  // namespace bjp
