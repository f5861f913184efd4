// Bandwidth references for the benchmark (not part of the solver): a pure
// read stream over a buffer, and random 8-byte gathers from a region of a
// given size.  They calibrate "achieved" figures against what this GPU's
// memory system delivers for the two access patterns the solver's kernels
// are made of (streamed tiles and CSR arrays; gathered vector entries).
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace {

constexpr int kThreads = 256;
typedef double v2d __attribute__((ext_vector_type(2)));

// Every thread streams 16-byte non-temporal loads, U in flight, over a
// grid-stride loop; one partial sum per workgroup keeps the loads live.
template <int U>
__global__ __launch_bounds__(kThreads) void k_read_stream(const v2d *buf, long long n2, double *out) {
    const long long stride = (long long)gridDim.x * kThreads;
    long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    double s = 0.0;
    for (; i + (U - 1) * stride < n2; i += U * stride) {
        v2d v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(buf + i + u * stride);
#pragma unroll
        for (int u = 0; u < U; ++u) s += v[u].x + v[u].y;
    }
    for (; i < n2; i += stride) {
        v2d a = __builtin_nontemporal_load(buf + i);
        s += a.x + a.y;
    }
    __shared__ double red[kThreads];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// count gathers of 8 bytes at pseudo-random places of src[0 .. 2^log2_elems):
// gather g reads src[(g * 0x9E3779B97F4A7C15) >> (64 - log2_elems)], eight in
// flight per thread.
__global__ __launch_bounds__(kThreads) void k_gather(const double *src, int log2_elems, long long count,
                                                     double *out) {
    const long long stride = (long long)gridDim.x * kThreads;
    const int sh = 64 - log2_elems;
    double s = 0.0;
    long long g = (long long)blockIdx.x * kThreads + threadIdx.x;
    for (; g + 7 * stride < count; g += 8 * stride) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const unsigned long long h = (unsigned long long)(g + u * stride) * 0x9E3779B97F4A7C15ull;
            v[u] = src[h >> sh];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; g < count; g += stride) s += src[((unsigned long long)g * 0x9E3779B97F4A7C15ull) >> sh];
    __shared__ double red[kThreads];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

}  // namespace

extern "C" {

// Read `bytes` (a multiple of 16, buf 16-byte aligned) once with `inflight`
// (4, 8 or 16) loads per thread in flight; out: device [grid] partial sums.
// Returns 0, or -1 for bad arguments.
int bjpcal_read_stream(const void *buf, size_t bytes, int grid, int inflight, double *out, hipStream_t stream) {
    if (!buf || !out || grid <= 0 || (bytes & 15) || (reinterpret_cast<uintptr_t>(buf) & 15)) return -1;
    const v2d *b = static_cast<const v2d *>(buf);
    const long long n2 = (long long)(bytes / 16);
    switch (inflight) {
        case 4: hipLaunchKernelGGL(k_read_stream<4>, dim3(grid), dim3(kThreads), 0, stream, b, n2, out); break;
        case 8: hipLaunchKernelGGL(k_read_stream<8>, dim3(grid), dim3(kThreads), 0, stream, b, n2, out); break;
        case 16: hipLaunchKernelGGL(k_read_stream<16>, dim3(grid), dim3(kThreads), 0, stream, b, n2, out); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// `count` random 8-byte gathers from src[0 .. 2^log2_elems); out: device
// [grid].  Returns 0, or -1 for bad arguments.
int bjpcal_gather(const double *src, int log2_elems, long long count, int grid, double *out, hipStream_t stream) {
    if (!src || !out || grid <= 0 || count < 0 || log2_elems < 1 || log2_elems > 40) return -1;
    hipLaunchKernelGGL(k_gather, dim3(grid), dim3(kThreads), 0, stream, src, log2_elems, count, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // extern "C"
