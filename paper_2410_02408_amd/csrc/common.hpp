// Shared device utilities for the block-Jacobi PCG library (gfx950, wave64).
//
// Reductions are deterministic: every workgroup reduces its values in a fixed
// tree and writes one partial per quantity; a one-workgroup finish kernel then
// sums the partials in a fixed order (no floating-point atomics).  The result
// does not depend on scheduling, and two runs on the same input are bitwise
// identical.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bjp.h"

namespace bjp {

constexpr int kWG = 256;             // threads per workgroup of the streaming kernels
constexpr int kWaves = kWG / 64;     // waves per workgroup
constexpr int kMaxRedWG = 2048;      // upper bound on workgroups that write partials
constexpr int kXcd = 8;              // MI355X: 8 XCDs, each with its own L2

// Workgroups are dispatched round-robin over the XCDs (workgroup b runs on XCD
// b % 8).  Remapping b to a chunk index so that each XCD owns one contiguous
// eighth of the data keeps neighbouring rows (stencil gathers, block tiles) in
// the same L2.  `grid` must be a multiple of 8.
__device__ __forceinline__ int xcd_chunk(int b, int grid) {
    return (b & (kXcd - 1)) * (grid / kXcd) + (b / kXcd);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Per-workgroup partial sums of NQ per-thread values: a fixed-order tree
// inside the workgroup, then thread 0 stores partials[q * gridDim.x + block].
// The totals are formed by a one-workgroup finish kernel launched next on the
// same stream (k_finish), so no workgroup needs a device-scope release fence:
// on gfx950 such a fence writes back the XCD's L2, and thousands of them per
// launch cost more than the launch itself.  Must be called by every thread.
template <int NQ>
__device__ __forceinline__ void block_partial(const double (&v)[NQ], double *partials) {
    __shared__ double red[NQ][kWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = wave_sum(v[q]);
        if (lane == 0) red[q][wave] = s;
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double s = 0.0;
            for (int w = 0; w < kWaves; ++w) s += red[q][w];
            partials[q * gridDim.x + blockIdx.x] = s;
        }
    }
}

// Per-workgroup partials stored at an explicit index (tile-indexed launches):
// partials[q * stride + index].
template <int NQ>
__device__ __forceinline__ void block_partial_at(const double (&v)[NQ], double *partials, int stride, int index) {
    __shared__ double red[NQ][kWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = wave_sum(v[q]);
        if (lane == 0) red[q][wave] = s;
    }
    __syncthreads();
    if (tid == 0 && index >= 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double s = 0.0;
            for (int w = 0; w < kWaves; ++w) s += red[q][w];
            partials[q * stride + index] = s;
        }
    }
}

// Sum of partials[q * stride + b] for b in [b0, b1), in a fixed order, for a
// one-workgroup launch; every thread receives the totals.
template <int NQ>
__device__ __forceinline__ void sum_partials_range(const double *partials, int stride, int b0, int b1,
                                                   double (&out)[NQ]) {
    __shared__ double red[NQ][kWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double acc = 0.0;
        for (int b = b0 + tid; b < b1; b += kWG) acc += partials[q * stride + b];
        acc = wave_sum(acc);
        if (lane == 0) red[q][wave] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w) s += red[q][w];
        out[q] = s;
    }
}

// This thread's share of the partials: partials[q * nparts + b] for
// b = tid, tid + 256, ..., summed in that order (nparts >= 1).  The loads of
// the first kMaxRedWG partials are issued before the first is used (clamped
// index, masked value; rounds past nparts are skipped for the whole
// workgroup).
template <int NQ>
__device__ __forceinline__ void thread_partials(const double *partials, int nparts, double (&acc)[NQ]) {
    constexpr int PER = kMaxRedWG / kWG;
    const int tid = threadIdx.x;
    double v[NQ][PER];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int j = 0; j < PER; ++j)
            v[q][j] = j * kWG < nparts ? partials[q * nparts + min(tid + j * kWG, nparts - 1)] : 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        acc[q] = 0.0;
#pragma unroll
        for (int j = 0; j < PER; ++j)
            if (tid + j * kWG < nparts) acc[q] += v[q][j];
        for (int b = tid + PER * kWG; b < nparts; b += kWG) acc[q] += partials[q * nparts + b];
    }
}

// Sum of partials[q * nparts + b] over b, in a fixed order, for a
// one-workgroup launch; every thread receives the totals.
template <int NQ>
__device__ __forceinline__ void sum_partials(const double *partials, int nparts, double (&out)[NQ]) {
    __shared__ double red[NQ][kWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double acc[NQ];
    thread_partials<NQ>(partials, nparts, acc);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        acc[q] = wave_sum(acc[q]);
        if (lane == 0) red[q][wave] = acc[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w) s += red[q][w];
        out[q] = s;
    }
}

// ---------------------------------------------------------------------------
// Device-resident solver state.  Written by thread 0 of one workgroup of a
// launch, read by every thread of the following launches.
// ---------------------------------------------------------------------------
struct PcgState {
    double rho;        // r^T z of the current iterate
    double alpha;      // rho / (p^T A p)
    double beta;       // rho_new / rho_old (0 after a (re)start)
    double bnorm2;     // ||b||^2
    double tol;        // relative residual target
    double relres;     // recursive ||r|| / ||b||
    double relres_true;
    int32_t it;        // completed iterations
    int32_t done;      // 1: stop iterating
    int32_t status;    // bjp_status
    int32_t max_iter;
    int32_t zero_rhs;  // b == 0
    int32_t pending;   // 1: the partials hold r^T z, r^T r of an update not yet decided
    int32_t xpend;     // 1: x += alpha p of the last step is not yet applied (done with
                       //    the next direction update, or by the solver at the end)
    int32_t pad;
};

struct LanczosState {
    double invb;       // 1 / beta of the vectors waiting to be normalised
    double beta_prev;  // beta_{j-1}
    double alpha_j;
    double scale;      // max |alpha|, beta seen so far
    double theta_min, theta_max, kappa;
    int32_t j;         // current step
    int32_t done;
    int32_t status;
    int32_t steps_done;
    int32_t steps;
    int32_t pad;
};

}  // namespace bjp
