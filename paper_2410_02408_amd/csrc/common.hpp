// Shared device utilities for the block-Jacobi PCG library (gfx950, wave64).
//
// Reductions are deterministic: every workgroup reduces its values in a fixed
// tree, writes one partial per quantity, and the last workgroup to arrive
// (integer arrival counter, no floating-point atomics) sums all partials in a
// fixed order.  The result therefore does not depend on scheduling, and two
// runs on the same input are bitwise identical.
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

__device__ __forceinline__ void store_agent(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_agent(const double *p) {
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide deterministic sum of NQ per-thread values.
//   partials: [NQ][gridDim.x] doubles, counter: one uint32 that is zero on
//   entry and is reset to zero by the last workgroup.
// Must be called by every thread of every workgroup of the launch.  Returns
// true in (every thread of) the last workgroup to arrive, where out[] holds
// the totals; other workgroups return false and out[] is unspecified.
template <int NQ>
__device__ __forceinline__ bool grid_sum(const double (&v)[NQ], double *partials,
                                         unsigned int *counter, double (&out)[NQ]) {
    __shared__ double red[NQ][kWaves];
    __shared__ int is_last;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int G = gridDim.x;
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
            store_agent(&partials[q * G + blockIdx.x], s);
        }
        __threadfence();
        unsigned int prev = atomicAdd(counter, 1u);
        is_last = (prev == (unsigned int)(G - 1));
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        acc[q] = 0.0;
        for (int b = tid; b < G; b += kWG) acc[q] += load_agent(&partials[q * G + b]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = wave_sum(acc[q]);
        if (lane == 0) red[q][wave] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w) s += red[q][w];
        out[q] = s;
    }
    if (tid == 0) atomicExch(counter, 0u);
    return true;
}

// ---------------------------------------------------------------------------
// Device-resident solver state.  Written only by the last workgroup of a
// launch (thread 0), read by every thread of the following launches.
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
    int32_t pad;
    unsigned int counter[4];
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
    unsigned int counter[4];
};

}  // namespace bjp
