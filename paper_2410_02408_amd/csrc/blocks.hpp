// Block-Jacobi preconditioner kernels: build (extract + Cholesky + inverse)
// and application z = M^-1 r.
//
// Storage of the block inverses ("diagonal packets").  A block of n <= G rows
// is handled by a group of G lanes (G = smallest power of two >= the largest
// block), so one wave of 64 lanes holds P = 64/G blocks: a packet.  Its
// symmetric inverse S (n x n) is stored by cyclic diagonals
//     d_k[i] = S[i][(i + k) mod n],   k = 0 .. floor(n/2),
// because d_{n-k} is d_k rotated, only half of the diagonals are needed:
// k = 0 .. G/2-1 are full rows of 64 scalars (one per lane of the packet), and
// for n = G the self-paired diagonal k = G/2 is a half row of 32 scalars.  A
// packet therefore holds 64*(G/2) + 32 scalars = P * G(G+1)/2, exactly the
// packed-triangle size.  Full diagonals are stored in pairs, interleaved per
// lane (diag_index): lane l reads d_k[l] and d_{k+1}[l] with one 16-byte load,
// so a wave's load covers 1 KB contiguously and a 64-row packet takes 17 loads
// per lane (16 pairs and the half row).  Blocks shorter than G use diagonals
// 0 .. floor(n/2) and zeros elsewhere.
//
// Application in lane i of a group:
//     z_i = sum_k d_k[i] r_{(i+k) mod n}              (upper part, own diagonal)
//         + sum_{0<k<n/2} d_k[(i-k) mod n] r_{(i-k) mod n}   (mirrored part)
// the first term rotates r across the group, the second moves the product
// d_k r computed by lane (i-k) to lane i; both are cross-lane permutes, so
// the tile never goes through LDS.
#pragma once

#include "common.hpp"
#include "finish.hpp"

namespace bjp {

__host__ __device__ constexpr int packet_elems(int G) { return G == 1 ? 64 : 64 * (G / 2) + 32; }

// Position in a packet of d_k for lane l = g*G + i (group g, row i): pairs
// (k, k+1), k even, interleaved per lane; an unpaired last full diagonal (G/2
// odd: G = 2) as a plain row; the half diagonal k = G/2 after the full ones.
__host__ __device__ constexpr int diag_index(int G, int k, int lane) {
    const int K = G / 2, Kp = K & ~1;
    return k < Kp ? (k >> 1) * 128 + 2 * lane + (k & 1)
                  : (k < K || K == 0 ? Kp * 64 + (k - Kp) * 64 + lane
                                     : K * 64 + (lane / G) * K + ((lane % G) & (K - 1)));
}

// Two scalars of the tile type, loaded or stored together.
template <typename TS>
struct Pair {
    typedef TS type __attribute__((ext_vector_type(2)));
};

// ---------------------------------------------------------------------------
// Build: one wave per packet.  LDS holds the P tiles (padded stride G+1).
// ---------------------------------------------------------------------------
struct SetupArgs {
    const int32_t *rp, *ci;
    const double *val;
    const int32_t *off;     // [nblocks+1]
    int nblocks;
    void *tiles;
    int32_t *flags;         // [0]: first failing block (INT_MAX if none)
    int block_base;         // added to the reported block index (batches)
};

// Setup of packet pk (one wave).  Kernel bodies of k_setup / k_setup_reg,
// shared with the batched setup, which finds each packet's system first.
template <int G, typename TS>
__device__ __forceinline__ void setup_lds_packet(const SetupArgs &a, int pk) {
    constexpr int P = 64 / G, LD = G + 1, E = packet_elems(G);
    __shared__ double T[P][G][LD];
    __shared__ double Wd[64];
    const int lane = threadIdx.x, g = lane / G, i = lane % G;
    const int t = pk * P + g;
    int s = 0, n = 0;
    if (t < a.nblocks) {
        s = a.off[t];
        n = a.off[t + 1] - s;
    }
    double (*Tg)[LD] = T[g];

    // 1. extract row s+i of the diagonal block (duplicates summed)
    for (int c = 0; c < G; ++c) Tg[i][c] = 0.0;
    if (i < n) {
        const int row = s + i;
        const int kb = a.rp[row], ke = a.rp[row + 1];
        for (int k = kb; k < ke; ++k) {
            const int c = a.ci[k] - s;
            if (c >= 0 && c < n) Tg[i][c] += a.val[k];
        }
    }
    __syncthreads();

    // 2. right-looking Cholesky A = L L^T, lane i owns row i
    bool ok = true;
    for (int j = 0; j < G; ++j) {
        const double d = (j < n) ? Tg[j][j] : 1.0;
        const double ljj = sqrt(d);
        if (i == j && j < n && !(d > 0.0 && isfinite(d))) ok = false;
        if (j < n && i > j && i < n) Tg[i][j] = Tg[i][j] / ljj;
        __syncthreads();
        if (j < n && i > j && i < n) {
            const double lij = Tg[i][j];
            for (int k = j + 1; k <= i; ++k) Tg[i][k] -= lij * Tg[k][j];
        }
        if (i == j && j < n) Tg[j][j] = ljj;
        __syncthreads();
    }
    if (!ok) atomicMin(&a.flags[0], a.block_base + t);

    // 3. W = L^-1 (lower); lane c computes column c, stored transposed in the
    //    strict upper triangle (W[k][c] at T[c][k]), diagonal 1/L_cc in Wd.
    if (i < n) Wd[g * G + i] = 1.0 / Tg[i][i];
    __syncthreads();
    for (int ii = 1; ii < G; ++ii) {
        if (i < ii && ii < n) {
            double acc = Wd[g * G + i] * Tg[ii][i];
            for (int k = i + 1; k < ii; ++k) acc += Tg[ii][k] * Tg[i][k];
            Tg[i][ii] = -acc * Wd[g * G + ii];
        }
    }
    __syncthreads();

    // 4. S = W^T W (= A_tt^-1); lane i computes S[i][j], j <= i, into the
    //    lower triangle (L is no longer needed).
    for (int j = 0; j < G; ++j) {
        if (j <= i && i < n) {
            double acc = Wd[g * G + i] * (i == j ? Wd[g * G + j] : Tg[j][i]);
            for (int k = i + 1; k < n; ++k) acc += Tg[i][k] * Tg[j][k];
            Tg[i][j] = acc;
        }
    }
    __syncthreads();

    // 5. store by cyclic diagonals (zeros where the block has no entry)
    TS *D = static_cast<TS *>(a.tiles) + (size_t)pk * E;
    const int nfull = (G == 1) ? 1 : G / 2;
    for (int k = 0; k < nfull; ++k) {
        double v = 0.0;
        if (i < n && 2 * k <= n) {
            int jj = i + k;
            if (jj >= n) jj -= n;
            v = (i >= jj) ? Tg[i][jj] : Tg[jj][i];
        }
        D[diag_index(G, k, lane)] = (TS)v;
    }
    if (G > 1 && i < G / 2) {
        double v = 0.0;
        if (n == G) v = Tg[i + G / 2][i];
        D[diag_index(G, G / 2, lane)] = (TS)v;
    }
}

template <int G, typename TS>
__global__ __launch_bounds__(64) void k_setup(SetupArgs a) {
    setup_lds_packet<G, TS>(a, blockIdx.x);
}

// Value of v in lane l (l wave-uniform).
__device__ __forceinline__ double lane_value(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Build with the rows held in registers (groups of G = 8 .. 64 lanes, P =
// 64/G blocks per wave): the same arithmetic as k_setup<G> in the same order
// (the stored inverses agree bit for bit up to the sign of exact zeros).
// Lane i of group g keeps row i of block g while it is factorised, then
// forms column i of L^-1 and multiplies it with the other columns.  What a
// step needs from other lanes (a pivot, a column of L, a row of L, the
// columns of L^-1) is read from a lane of the group (readlane for one group
// per wave, a permute otherwise) or written to LDS once and read back by the
// group at one address (a broadcast), all of a step's reads issued before
// its arithmetic; the loops over columns are unrolled so every register
// index is a compile-time constant.  Rows past a block's end are set to the
// identity, which leaves the block's own entries unchanged (its couplings to
// them are zero) and keeps bounds tests out of the unrolled loops.  Measured
// at 128^3, n_b = 64: 1.7 ms instead of 9.3 ms for the 32,768 blocks.
template <int G, typename TS>
__device__ __forceinline__ void setup_reg_packet(const SetupArgs &a, int pk) {
    static_assert(G >= 8 && G <= 64 && (G & (G - 1)) == 0, "paired diagonals need G / 2 even");
    constexpr int P = 64 / G, LDM = G + 2, E = packet_elems(G);   // LDM: 16-byte aligned rows
    __shared__ __align__(16) double Mx[64][LDM];
    __shared__ __align__(16) double cb[2][64];
    __shared__ double Wd[64];
    const int lane = threadIdx.x, g = lane / G, i = lane % G, base = g * G;
    const int t = pk * P + g;
    int s = 0, n = 0;
    if (t < a.nblocks) {
        s = a.off[t];
        n = a.off[t + 1] - s;
    }

    // 1. extract row s + i of the diagonal block (duplicates summed)
#pragma unroll
    for (int c = 0; c < G; ++c) Mx[lane][c] = 0.0;
    if (i < n) {
        const int row = s + i;
        const int kb = a.rp[row], ke = a.rp[row + 1];
        for (int k = kb; k < ke; ++k) {
            const int c = a.ci[k] - s;
            if (c >= 0 && c < n) Mx[lane][c] += a.val[k];
        }
    } else {
        Mx[lane][i] = 1.0;
    }
    double r[G];
#pragma unroll
    for (int c = 0; c < G; ++c) r[c] = Mx[lane][c];

    // 2. right-looking Cholesky: step j takes the pivot from row j, scales
    //    column j below it and updates the trailing rows (i > j) with column
    //    j broadcast through LDS
    bool bad = false;
#pragma unroll
    for (int j = 0; j < G; ++j) {
        double d;
        if constexpr (G == 64) d = lane_value(r[j], j);
        else d = __shfl(r[j], base + j, 64);
        if (j < n && !(d > 0.0 && isfinite(d))) bad = true;
        const double ljj = sqrt(d);
        if (i > j) r[j] = r[j] / ljj;
        if (i == j) r[j] = ljj;
        if (j + 1 < G) {
            double *col = cb[j & 1] + base;
            col[i] = r[j];
            __syncthreads();
            double cv[G];
#pragma unroll
            for (int k = j + 1; k < G; ++k) cv[k] = col[k];
            __builtin_amdgcn_sched_barrier(0);
            if (i > j) {
#pragma unroll
                for (int k = j + 1; k < G; ++k) r[k] -= r[j] * cv[k];
            }
        }
    }
    if (bad && i == 0) atomicMin(&a.flags[0], a.block_base + t);

    // 3. W = L^-1 by columns: lane i forms W[ii][i] row by row from row ii
    //    of L (broadcast); W[i][i] = 1 / L[i][i], zeros above
#pragma unroll
    for (int c = 0; c < G; ++c) Mx[lane][c] = r[c];
    Wd[lane] = 1.0 / Mx[lane][i];
    __syncthreads();
    double w[G];
    {
        const double wself = Wd[lane];
#pragma unroll
        for (int k = 0; k < G; ++k) w[k] = (k == i) ? wself : 0.0;
    }
#pragma unroll
    for (int ii = 1; ii < G; ++ii) {
        double lv[G];
#pragma unroll
        for (int k = 0; k < ii; ++k) lv[k] = Mx[base + ii][k];
        const double wd = Wd[base + ii];
        __builtin_amdgcn_sched_barrier(0);
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < ii; ++k) acc += lv[k] * w[k];
        if (i < ii) w[ii] = -acc * wd;
    }
    __syncthreads();

    // 4. S = W^T W by cyclic diagonals: d_k[i] = S[i][(i+k) mod n] is column
    //    i of W (this lane) against column (i+k) mod n (from LDS); stored in
    //    the packet's interleaved pairs, zeros outside the block
#pragma unroll
    for (int m = 0; m < G; ++m) Mx[lane][m] = w[m];
    __syncthreads();
    TS *D = static_cast<TS *>(a.tiles) + (size_t)pk * E;
    typedef typename Pair<TS>::type TS2;
    auto diag = [&](int k) -> double {
        if (i >= n || 2 * k > n) return 0.0;
        int jj = i + k;
        if (jj >= n) jj -= n;
        double wv[G];
#pragma unroll
        for (int m = 0; m < G; ++m) wv[m] = Mx[base + jj][m];
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < G; ++m) acc += w[m] * wv[m];
        return acc;
    };
    for (int k = 0; k < G / 2; k += 2) {
        TS2 v;
        v.x = (TS)diag(k);
        v.y = (TS)diag(k + 1);
        *reinterpret_cast<TS2 *>(D + diag_index(G, k, lane)) = v;
    }
    if (i < G / 2) {
        double v = 0.0;
        if (n == G) {
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < G; ++m) acc += w[m] * Mx[base + i + G / 2][m];
            v = acc;
        }
        D[diag_index(G, G / 2, lane)] = (TS)v;
    }
}

template <int G, typename TS>
__global__ __launch_bounds__(64) void k_setup_reg(SetupArgs a) {
    setup_reg_packet<G, TS>(a, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Application
// ---------------------------------------------------------------------------
#ifndef BJP_NT_TILES
#define BJP_NT_TILES 1
#endif

// Tile loads: the packets are streamed once per application and exceed every
// cache level, so they are loaded non-temporally (the vectors' lines stay
// cached; measured at 128^3, n_b = 64 with the unpipelined loop: 130 us
// instead of 145 us per application).
template <typename TS>
__device__ __forceinline__ TS tile_load(const TS *p) {
#if BJP_NT_TILES
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

// One packet, one wave: lane i of group g holds row i of block g.
// packet_load issues the K + 1 loads of this lane's diagonal entries (the
// half row counts as diagonal K = G/2); packet_product forms z_i from them.

template <int G, typename TS>
__device__ __forceinline__ void packet_load(const TS *__restrict__ D, int lane, int g, int i, TS (&dv)[G / 2 + 1]) {
    constexpr int K = G / 2, Kp = K & ~1;
    typedef typename Pair<TS>::type TS2;
#pragma unroll
    for (int k = 0; k < Kp; k += 2) {
        const TS2 v = tile_load(reinterpret_cast<const TS2 *>(D + diag_index(G, k, lane)));
        dv[k] = v.x;
        dv[k + 1] = v.y;
    }
#pragma unroll
    for (int k = Kp; k <= K; ++k) dv[k] = tile_load(D + diag_index(G, k, lane));
}

// Whole-wave rotations by one lane (DPP): kDppWaveRor1 gives lane i the
// value of lane i-1, kDppWaveRol1 that of lane i+1 (lane indices mod 64).
constexpr int kDppWaveRol1 = 0x134, kDppWaveRor1 = 0x13C;

// (every lane is written, so no previous value of the destination is kept)
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

// z = S r for one full 64 x 64 block held as cyclic diagonals dv[0..32]
// (dv[32] is the half diagonal: lanes i and i + 32 hold the same entry).
//   direct part      sum_k d_k[i] r[i+k]        k = 0 .. 32
//   transposed part  sum_k d_k[i-k] r[i-k]      k = 1 .. 31
// r[i+k] comes from k successive one-lane rotations of r; the transposed part
// is evaluated Horner-style, acc_k = d_k r + (acc_{k+1} moved up one lane),
// so only one-lane rotations are needed and no lane index is computed.
template <typename TS>
__device__ __forceinline__ TS full64_product(const TS (&dv)[33], TS rs) {
    TS zd = dv[0] * rs;
    TS rr = rs;
#pragma unroll
    for (int k = 1; k <= 32; ++k) {
        rr = dpp_move<kDppWaveRol1>(rr);
        zd += dv[k] * rr;
    }
    TS acc = dv[31] * rs;
#pragma unroll
    for (int k = 30; k >= 1; --k) acc = dv[k] * rs + dpp_move<kDppWaveRor1>(acc);
    return zd + dpp_move<kDppWaveRor1>(acc);
}

// Any block size n <= G: entries are addressed modulo n, lanes i >= n and
// the wrapped half of the middle diagonal are masked.  Full 64-row blocks
// take the rotation form above.
template <int G, typename TS>
__device__ __forceinline__ TS packet_product(const TS (&dv)[G / 2 + 1], int g, int i, int n, TS rs) {
    constexpr int K = G / 2;
    if constexpr (G == 64) {
        if (__builtin_amdgcn_readfirstlane(n) == 64) return full64_product<TS>(dv, rs);
    }
    const bool act = i < n;
    const int ia = act ? i : 0;
    const int nn = n > 0 ? n : 1;
    TS zv = dv[0] * rs;
#pragma unroll
    for (int k = 1; k <= K; ++k) {
        int j1 = ia + k;
        if (j1 >= nn) j1 -= nn;
        int j2 = ia - k;
        if (j2 < 0) j2 += nn;
        const TS rk = __shfl(rs, g * G + (j1 & (G - 1)), 64);
        if (act && 2 * k <= n) zv += dv[k] * rk;
        const TS tv = (act && 2 * k < n) ? dv[k] * rs : (TS)0;
        const TS tt = __shfl(tv, g * G + (j2 & (G - 1)), 64);
        if (act && 2 * k < n) zv += tt;
    }
    return zv;
}

// UPDATE: x += alpha p, r -= alpha q, z = M^-1 r (the batched solver);
// STEP: r -= alpha q, z = M^-1 r (the single-system solver applies the x
// update in the next direction update).
enum ApplyMode { APPLY_PLAIN = 0, APPLY_INIT = 1, APPLY_UPDATE = 2, APPLY_LANCZOS = 3, APPLY_STEP = 4 };

struct ApplyArgs {
    int nblocks, num_packets;
    int n;                  // rows of the system
    int row0;               // first row of the system (0 except in batches)
    int uniform_nb;         // > 0: block t = rows [row0 + t*nb, ...), offsets unused
    const int32_t *off;
    const void *tiles;
    const double *rin;      // PLAIN / INIT / LANCZOS: residual to precondition
    double *zout;           // PLAIN / INIT / LANCZOS / UPDATE: z = M^-1 r
    PcgState *st;           // INIT / UPDATE (UPDATE: the state after the direction update)
    PcgState *st_out;       // UPDATE: where workgroup 0 records the state with alpha
    const double *dec_partials;  // UPDATE: partials of p^T A p from the product
    int dec_nparts;
    double *x, *r;          // UPDATE: x += alpha p, r -= alpha q
    const double *q;
    double *p0, *p1;        // UPDATE: p_new = p[(it+1)&1]
    LanczosState *ls;       // LANCZOS
    double *partials;       // per-workgroup r^T z, r^T r
};

// Packets pk0, pk0 + stride, ... < pk1 of one system (rows [a.row0,
// a.row0 + a.n), tiles at a.tiles) in the given mode; accumulates this
// thread's share of r^T z and r^T r.  One wave per packet.  `st` gives the
// iteration count (the direction buffer); pre(alpha), called by every thread
// once the first packet's loads are issued, supplies the step length and
// returns false to skip the work.
template <int G, typename TS, int MODE, typename Pre>
__device__ __forceinline__ void apply_packets(const ApplyArgs &a, const PcgState *st, int pk0, int pk1, int stride,
                                              double &d0, double &d1, Pre pre) {
    constexpr int P = 64 / G, E = packet_elems(G);
    const int lane = threadIdx.x & 63;
    const int g = lane / G, i = lane % G;
    double alpha = 0.0;
    const double *__restrict__ pn = nullptr;
    if (MODE == APPLY_UPDATE) pn = ((st->it + 1) & 1) ? a.p1 : a.p0;
    const TS *__restrict__ tiles = static_cast<const TS *>(a.tiles);
    const int32_t *__restrict__ off = a.off;
    double *__restrict__ xv_ = a.x;
    double *__restrict__ rv_ = a.r;
    const double *__restrict__ qv_ = a.q;
    const double *__restrict__ rin = a.rin;
    double *__restrict__ zout = a.zout;
    const int rend = a.row0 + a.n;
    // Two stages in turn: while the packet of one stage is multiplied, the
    // loads of the next packet fill the other.  Unrolled by two so that no
    // register copy (which would wait for the pending loads) is needed.
    constexpr int NV = MODE == APPLY_UPDATE ? 4 : MODE == APPLY_STEP ? 2 : 1;
    constexpr int ND = G / 2 + 1;
    struct Stage {
        TS d[ND];
        double v[NV];
        int s, n;
    };
    auto stage_load = [&](Stage &S, int pk) {
        const int t = pk * P + g;
        if (a.uniform_nb > 0) {
            S.s = a.row0 + t * a.uniform_nb;
            S.n = max(0, min(a.uniform_nb, rend - S.s));
        } else {
            const int tc = min(t, a.nblocks - 1);
            const int s0 = off[tc], e0 = off[tc + 1];
            S.s = t < a.nblocks ? s0 : 0;
            S.n = t < a.nblocks ? e0 - s0 : 0;
        }
        const int rc = min(S.s + i, rend - 1);    // in-bounds index for masked lanes
        if constexpr (MODE == APPLY_UPDATE) {
            S.v[0] = xv_[rc];
            S.v[1] = pn[rc];
            S.v[2] = qv_[rc];
            S.v[3] = rv_[rc];
        } else if constexpr (MODE == APPLY_STEP) {
            // r is next read by the next application, after every tile has
            // streamed through the caches: read and written non-temporally
            // (measured at 128^3: 0.7 us per iteration)
            S.v[0] = qv_[rc];
            S.v[1] = __builtin_nontemporal_load(rv_ + rc);
        } else {
            S.v[0] = rin[rc];
        }
        packet_load<G, TS>(tiles + (size_t)pk * E, lane, g, i, S.d);
    };
    auto stage_apply = [&](const Stage &S) {
        const bool act = i < S.n;
        const int row = S.s + i;
        double rv;
        if constexpr (MODE == APPLY_UPDATE) {
            rv = act ? fma(-alpha, S.v[2], S.v[3]) : 0.0;
        } else if constexpr (MODE == APPLY_STEP) {
            rv = act ? fma(-alpha, S.v[0], S.v[1]) : 0.0;
        } else {
            rv = act ? S.v[0] : 0.0;
        }
        const TS zv = packet_product<G, TS>(S.d, g, i, S.n, (TS)rv);
        if (act) {
            if constexpr (MODE == APPLY_UPDATE) {
                xv_[row] = fma(alpha, S.v[1], S.v[0]);
                rv_[row] = rv;
            } else if constexpr (MODE == APPLY_STEP) {
                __builtin_nontemporal_store(rv, rv_ + row);
            }
            const double z = (double)zv;
            zout[row] = z;
            d0 += rv * z;
            d1 += rv * rv;
        }
    };
    const bool any = pk0 < pk1;
    Stage A, B;
    if (any) stage_load(A, pk0);
    if (!pre(alpha) || !any) return;
    for (int pk = pk0;;) {
        // past the end the current packet is loaded again: loads stay in bounds
        stage_load(B, pk + stride < pk1 ? pk + stride : pk);
        __builtin_amdgcn_sched_barrier(0);
        stage_apply(A);
        pk += stride;
        if (pk >= pk1) break;
        stage_load(A, pk + stride < pk1 ? pk + stride : pk);
        __builtin_amdgcn_sched_barrier(0);
        stage_apply(B);
        pk += stride;
        if (pk >= pk1) break;
    }
}

// STEP first takes the step-length decision alpha = rho / (p^T A p) in
// every workgroup (from the product's partials), then updates r, applies
// M^-1 and marks the update decision pending for the next launch.  Wave w of
// the launch takes packets w, w + W, w + 2W, ... (W waves in all), so the
// whole launch streams one contiguous window of the packed inverses at a
// time (measured at 128^3, n_b = 64: 1.7 us per application faster than
// contiguous runs of packets per workgroup).
template <int G, typename TS, int MODE>
__global__ __launch_bounds__(kWG) void k_apply(ApplyArgs a) {
    if (MODE == APPLY_INIT) {
        if (a.st->done) return;
    }
    if (MODE == APPLY_LANCZOS) {
        if (a.ls->done) return;
    }
    const int wave = threadIdx.x >> 6;
    double d0 = 0.0, d1 = 0.0;
    auto pre = [&](double &alpha) -> bool {
        if (MODE != APPLY_STEP) return true;
        const PcgState L = shared_decide<FIN_SIGMA>(a.st, a.st_out, a.dec_partials, a.dec_nparts, nullptr, true);
        alpha = L.alpha;
        return !L.done;
    };
    apply_packets<G, TS, MODE>(a, a.st, blockIdx.x * kWaves + wave, a.num_packets, gridDim.x * kWaves, d0, d1, pre);
    if (MODE == APPLY_PLAIN) return;
    const double v[2] = {d0, d1};
    block_partial<2>(v, a.partials);
}

// Preconditioner-free (M = I) counterpart of k_apply for PCG: z is r itself
// (modes INIT and STEP).
template <int MODE>
__global__ __launch_bounds__(kWG) void k_rows_update(ApplyArgs a, int n, int chunk) {
    double alpha = 0.0;
    if (MODE == APPLY_STEP) {
        const PcgState L = shared_decide<FIN_SIGMA>(a.st, a.st_out, a.dec_partials, a.dec_nparts, nullptr, true);
        if (L.done) return;
        alpha = L.alpha;
    } else if (a.st->done) {
        return;
    }
    const int c = xcd_chunk(blockIdx.x, gridDim.x);
    const int r0 = c * chunk, r1 = min(r0 + chunk, n);
    double d1 = 0.0;
    for (int row = r0 + threadIdx.x; row < r1; row += kWG) {
        double rv = a.r[row];
        if (MODE == APPLY_STEP) {
            rv = fma(-alpha, a.q[row], rv);
            a.r[row] = rv;
        }
        d1 += rv * rv;
    }
    const double v[1] = {d1};
    block_partial<1>(v, a.partials);
}

}  // namespace bjp
