// Batched block-Jacobi PCG: many independent systems, each launch covering
// all of them.
//
// The batch is one block-diagonal CSR matrix (system s owns rows
// [row0_s, row0_s + n_s) and its columns stay inside that range) with a block
// size per system.  Work is cut into tiles that never straddle two systems:
//   row tiles    (s, r0, r1)   for the SpMV and the direction update,
//   packet tiles (s, pk0, pk1) for the block-inverse application, grouped by
//                              the system's lane-group width G (one launch per
//                              width present in the batch).
// Every system carries its own PcgState; each tile skips its work when its
// system is done, and a one-workgroup-per-system finish kernel takes the
// same scalar decisions as the single-system solver from the partial sums of
// that system's tiles.  All systems therefore advance together, one
// iteration per sequence of launches, and a converged system costs only the
// state check of its tiles.
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

struct Tile {
    int s, a0, a1, pad;   // system, first and end row (or packet)
};

struct TileSpan {
    const Tile *tiles;
    int begin, end;       // tiles [begin, end) of the table are this launch's
    int stride;           // partials are laid out [q][stride]
    const SysInfo *sys;
};

// Workgroup b of a tile launch handles tile begin + xcd_chunk(b) (the grid is
// a multiple of 8; workgroups past the end only take part in the reduction
// tree and store nothing).
__device__ __forceinline__ int tile_of(const TileSpan &ts) {
    return ts.begin + xcd_chunk(blockIdx.x, gridDim.x);
}

// The batch's block setup, one launch per lane-group width: workgroup q
// takes packet q of the width's systems taken in order; items[] lists those
// systems with the index of each one's first packet (ascending).
struct SetupSys {
    long long off_base;   // index of the system's first block offset
    long long tile0;      // first scalar of the system's packets
    int nblocks, block_base, first_packet, pad;
};

template <int G, typename TS>
__global__ __launch_bounds__(64) void k_setup_batch(SetupArgs base, const SetupSys *items, int count) {
    const int q = blockIdx.x;
    int lo = 0, hi = count - 1;   // the last system whose first packet is <= q
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].first_packet <= q) lo = mid;
        else hi = mid - 1;
    }
    SetupArgs a = base;
    a.off = base.off + items[lo].off_base;
    a.nblocks = items[lo].nblocks;
    a.tiles = static_cast<TS *>(base.tiles) + items[lo].tile0;
    a.block_base = items[lo].block_base;
    const int pk = q - items[lo].first_packet;
    if constexpr (G >= 8) setup_reg_packet<G, TS>(a, pk);
    else setup_lds_packet<G, TS>(a, pk);
}

template <int GS, int MODE>
__global__ __launch_bounds__(kWG) void k_spmv_tiles(SpmvArgs a, TileSpan ts) {
    const int t = tile_of(ts);
    double d0 = 0.0, d1 = 0.0;
    if (t < ts.end) {
        const Tile tl = ts.tiles[t];
        const PcgState *st = a.st + tl.s;
        const bool run = (MODE == SPMV_RESID && a.resid_phase == 1) || !st->done;
        if (run) spmv_rows<GS, MODE>(a, st->it, tl.a0, tl.a1, d0, d1);
    }
    const double v[2] = {d0, d1};
    block_partial_at<2>(v, a.partials, ts.stride, t < ts.end ? t : -1);
}

// Row-block streaming schedule over row tiles (short rows); CSR loads are
// non-temporal (the batch's matrix exceeds the last-level cache).
template <int MODE>
__global__ __launch_bounds__(kWG) void k_spmv_tiles_stream(SpmvArgs a, TileSpan ts) {
    const int t = tile_of(ts);
    double d0 = 0.0, d1 = 0.0;
    __shared__ double prod[kStreamPer * kWG];
    if (t < ts.end) {
        const Tile tl = ts.tiles[t];
        const PcgState *st = a.st + tl.s;
        const bool run = (MODE == SPMV_RESID && a.resid_phase == 1) || !st->done;
        if (run) spmv_stream_rows<MODE, true>(a, st->it, tl.a0, tl.a1, d0, d1, prod);
    }
    const double v[2] = {d0, d1};
    block_partial_at<2>(v, a.partials, ts.stride, t < ts.end ? t : -1);
}

template <int G, typename TS, int MODE>
__global__ __launch_bounds__(kWG) void k_apply_tiles(ApplyArgs a, TileSpan ts) {
    const int t = tile_of(ts);
    double d0 = 0.0, d1 = 0.0;
    if (t < ts.end) {
        const Tile tl = ts.tiles[t];
        const PcgState *st = a.st + tl.s;
        if (!st->done) {
            const SysInfo si = ts.sys[tl.s];
            ApplyArgs b = a;
            b.row0 = si.row0;
            b.n = si.n;
            b.uniform_nb = si.nb;
            b.nblocks = si.nblocks;
            b.tiles = static_cast<const TS *>(a.tiles) + si.tile0;
            auto pre = [&](double &alpha) -> bool {
                if (MODE == APPLY_UPDATE) alpha = st->alpha;
                return true;
            };
            apply_packets<G, TS, MODE>(b, st, tl.a0 + (threadIdx.x >> 6), tl.a1, kWaves, d0, d1, pre);
        }
    }
    const double v[2] = {d0, d1};
    block_partial_at<2>(v, a.partials, ts.stride, t < ts.end ? t : -1);
}

// Start of a batch solve from x = 0, over the row tiles: x cleared, r = b
// (b - A x with x = 0) and the partials the residual product would leave.
__global__ __launch_bounds__(kWG) void k_start_zero_tiles(const double *b, double *x, double *r, double *partials,
                                                          TileSpan ts) {
    const int t = tile_of(ts);
    double d = 0.0;
    if (t < ts.end) {
        const Tile tl = ts.tiles[t];
        for (int i = tl.a0 + threadIdx.x; i < tl.a1; i += kWG) {
            const double v = b[i];
            x[i] = 0.0;
            r[i] = v;
            d += v * v;
        }
    }
    const double v[2] = {d, d};
    block_partial_at<2>(v, partials, ts.stride, t < ts.end ? t : -1);
}

// p_new = z + beta_s p_old over the rows of each active system.
__global__ __launch_bounds__(kWG) void k_direction_tiles(PcgState *states, const double *z, double *p0,
                                                         double *p1, TileSpan ts) {
    const int t = tile_of(ts);
    if (t >= ts.end) return;
    const Tile tl = ts.tiles[t];
    const PcgState *st = states + tl.s;
    if (st->done) return;
    const int it = st->it;
    const double *pold = (it & 1) ? p1 : p0;
    double *pnew = (it & 1) ? p0 : p1;
    const double beta = st->beta;
    for (int i = tl.a0 + threadIdx.x; i < tl.a1; i += kWG) pnew[i] = dir_value(beta, pold, z, i);
}

__global__ void k_batch_state_init(PcgState *states, int S, double tol, const int *max_iter) {
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < S; s += gridDim.x * blockDim.x) {
        PcgState st{};
        st.tol = tol;
        st.max_iter = max_iter[s];
        st.status = BJP_OK;
        states[s] = st;
    }
}

// Re-open the listed systems after a failed true-residual check (residual
// replacement): the direction restarts from r = b - A x.
__global__ void k_batch_restart(PcgState *states, const int *list, int count) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < count; k += gridDim.x * blockDim.x) {
        PcgState *st = states + list[k];
        st->done = 0;
        st->status = BJP_OK;
    }
}

// Every column of a row must lie in the row's own system.  A system's rows
// are contiguous, so its entries are the contiguous range rp[lo] .. rp[hi] of
// ci (row_ptr has been validated before this launch): one workgroup per
// system scans that range coalesced, four loads in flight per thread.
__global__ __launch_bounds__(kWG) void k_validate_batch(int S, const int32_t *sys_rows, const int32_t *rp,
                                                        const int32_t *ci, int32_t *flags) {
    for (int s = blockIdx.x; s < S; s += gridDim.x) {
        const int lo = sys_rows[s], hi = sys_rows[s + 1];
        const int e0 = rp[lo], e1 = rp[hi];
        bool bad = false;
        int k = e0 + threadIdx.x;
        for (; k + 3 * kWG < e1; k += 4 * kWG) {
            const int c0 = ci[k], c1 = ci[k + kWG], c2 = ci[k + 2 * kWG], c3 = ci[k + 3 * kWG];
            bad |= c0 < lo || c0 >= hi || c1 < lo || c1 >= hi || c2 < lo || c2 >= hi || c3 < lo || c3 >= hi;
        }
        for (; k < e1; k += kWG) {
            const int c = ci[k];
            bad |= c < lo || c >= hi;
        }
        if (bad) atomicOr(&flags[1], 1);
    }
}

}  // namespace bjp
