// Host side of the C ABI declared in include/bjp.h: argument checks,
// workspace carving, launch configuration and the PCG / Lanczos drivers.
// The library allocates no device memory; every buffer lives in the caller's
// workspace.  All launches go to the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "adjoint.hpp"
#include "batch.hpp"
#include "bjp.h"
#include "blocks.hpp"
#include "common.hpp"
#include "finish.hpp"
#include "lanczos.hpp"
#include "small.hpp"
#include "spmv.hpp"

using namespace bjp;

namespace {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }
inline int round8(int g) { return std::max(8, (g + 7) & ~7); }
inline int pow2_at_least(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

#define HIP_TRY(expr)                                 \
    do {                                              \
        if ((expr) != hipSuccess) return BJP_EHIP;    \
    } while (0)

struct Carver {
    char *base;
    size_t used = 0;
    template <typename T>
    T *take(size_t count) {
        T *p = reinterpret_cast<T *>(base + used);
        used += al256(count * sizeof(T));
        return p;
    }
};

int check_csr_host(const bjp_csr_t *A) {
    if (!A || A->n < 0 || A->nnz < 0 || A->n > BJP_MAX_DIM || A->nnz > BJP_MAX_DIM) return BJP_EINVAL;
    if (A->n > 0 && !A->row_ptr) return BJP_EINVAL;
    if (A->nnz > 0 && (!A->col_idx || !A->val)) return BJP_EINVAL;
    return BJP_OK;
}

// ---------------------------------------------------------------------------
// utility kernels
// ---------------------------------------------------------------------------
__global__ void k_fill(double *p, int n, double v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// off[t] = t * nb for t < nblocks, off[nblocks] = n.
__global__ void k_uniform_offsets(int32_t *off, int nblocks, int nb, int n) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t <= nblocks; t += gridDim.x * blockDim.x)
        off[t] = t == nblocks ? n : (int32_t)((long long)t * nb);
}

__global__ void k_fill_i32(int32_t *p, int n, int32_t v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_flags_init(int32_t *flags) {
    if (threadIdx.x == 0) {
        flags[0] = INT_MAX;
        flags[1] = 0;
        flags[2] = 0;
        flags[3] = 0;
    }
}

// flags[1] |= structural error, flags[2] |= non-finite value
__global__ void k_validate(int n, int nnz, const int32_t *rp, const int32_t *ci, const double *val,
                           int32_t *flags) {
    const int stride = gridDim.x * blockDim.x;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false, nonfinite = false;
    for (int i = g; i < n; i += stride) {
        const int b = rp[i], e = rp[i + 1];
        if (b < 0 || e < b || e > nnz) bad = true;
        if (i == 0 && b != 0) bad = true;
        if (i == n - 1 && e != nnz) bad = true;
    }
    for (int k = g; k < nnz; k += stride) {
        const int c = ci[k];
        if (c < 0 || c >= n) bad = true;
        if (!isfinite(val[k])) nonfinite = true;
    }
    if (bad) atomicOr(&flags[1], 1);
    if (nonfinite) atomicOr(&flags[2], 1);
}

__global__ void k_pcg_state_init(PcgState *st, double tol, int max_iter) {
    if (threadIdx.x != 0) return;
    st->rho = st->alpha = st->beta = 0.0;
    st->bnorm2 = 0.0;
    st->tol = tol;
    st->relres = st->relres_true = 0.0;
    st->it = 0;
    st->done = 0;
    st->status = BJP_OK;
    st->max_iter = max_iter;
    st->zero_rhs = 0;
    st->pending = 0;
    st->xpend = 0;
    st->pad = 0;
}

__global__ void k_pcg_restart(PcgState *st) {
    if (threadIdx.x == 0) {
        st->done = 0;
        st->status = BJP_OK;
    }
}

__global__ void k_lanczos_state_init(LanczosState *ls, int steps) {
    if (threadIdx.x != 0) return;
    ls->invb = ls->beta_prev = ls->alpha_j = ls->scale = 0.0;
    ls->theta_min = ls->theta_max = ls->kappa = 0.0;
    ls->j = 0;
    ls->done = 0;
    ls->status = BJP_OK;
    ls->steps_done = 0;
    ls->steps = steps;
    ls->pad = 0;
}

// Lanczos start: partial r^T z for z = M^-1 r (z == r when M = I); the
// finish kernel turns it into 1 / beta_0.
__global__ __launch_bounds__(kWG) void k_lanczos_start(LanczosState *ls, const double *r,
                                                       const double *z, int n, int chunk,
                                                       double *partials) {
    if (ls->done) return;
    const int c = xcd_chunk(blockIdx.x, gridDim.x);
    const int r0 = c * chunk, r1 = min(r0 + chunk, n);
    double s = 0.0;
    for (int i = r0 + threadIdx.x; i < r1; i += kWG) s += r[i] * z[i];
    const double v[1] = {s};
    block_partial<1>(v, partials);
}

template <int OP>
void finish(const FinishArgs &f, int nparts, hipStream_t s) {
    FinishArgs g = f;
    g.nparts = nparts;
    hipLaunchKernelGGL((k_finish<OP>), dim3(1), dim3(kWG), 0, s, g);
}

// ---------------------------------------------------------------------------
// partition
// ---------------------------------------------------------------------------
// Uniform partitions keep no host copy of their offsets (the device forms
// them); explicit ones are copied from the caller.
struct Partition {
    std::vector<int32_t> off;   // explicit partitions: nblocks + 1 offsets
    int uniform = 0;            // > 0: blocks of `uniform` rows, last one ragged
    int nblocks = 0, G = 1, packets = 0, E = 64;
};

int make_partition(int n, const bjp_block_spec_t *spec, Partition &P) {
    if (!spec) return BJP_EINVAL;
    P.off.clear();
    P.uniform = 0;
    if (spec->block_size > 0) {
        if (spec->block_size > BJP_MAX_BLOCK) return BJP_EINVAL;
        // a block size above n gives one block of n rows
        P.uniform = n > 0 ? std::min(spec->block_size, n) : spec->block_size;
        P.nblocks = ceil_div(n, P.uniform);
        P.G = pow2_at_least(n > 0 ? P.uniform : 1);
        P.packets = ceil_div(P.nblocks, 64 / P.G);
        P.E = packet_elems(P.G);
        return BJP_OK;
    } else if (spec->block_size == 0) {
        if (spec->num_blocks < 0 || !spec->offsets) return BJP_EINVAL;
        P.off.assign(spec->offsets, spec->offsets + spec->num_blocks + 1);
        if (P.off.front() != 0 || P.off.back() != n) return BJP_EINVAL;
        for (int t = 0; t < spec->num_blocks; ++t) {
            const int m = P.off[t + 1] - P.off[t];
            if (m <= 0 || m > BJP_MAX_BLOCK) return BJP_EINVAL;
        }
    } else {
        return BJP_EINVAL;
    }
    P.nblocks = (int)P.off.size() - 1;
    int maxb = 1;
    for (int t = 0; t < P.nblocks; ++t) maxb = std::max(maxb, P.off[t + 1] - P.off[t]);
    P.G = pow2_at_least(maxb);
    P.packets = ceil_div(P.nblocks, 64 / P.G);
    P.E = packet_elems(P.G);
    return BJP_OK;
}

size_t precond_ws_bytes(const Partition &P, int precision) {
    const size_t s = precision == BJP_FP32_STORE ? 4 : 8;
    return al256(sizeof(int32_t) * ((size_t)P.nblocks + 1)) + al256((size_t)P.packets * P.E * s) + al256(64);
}

int run_validate(const bjp_csr_t *A, int32_t *flags, hipStream_t stream) {
    hipLaunchKernelGGL(k_flags_init, dim3(1), dim3(64), 0, stream, flags);
    if (A->n > 0 || A->nnz > 0) {
        const int work = std::max(A->n, A->nnz);
        const int grid = std::min(ceil_div(work, kWG), 4096);
        hipLaunchKernelGGL(k_validate, dim3(std::max(grid, 1)), dim3(kWG), 0, stream, A->n, A->nnz,
                           A->row_ptr, A->col_idx, A->val, flags);
    }
    HIP_TRY(hipGetLastError());
    int32_t h[4];
    HIP_TRY(hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (h[1]) return BJP_EINVAL;
    if (h[2]) return BJP_ENONFINITE;
    return BJP_OK;
}

// ---------------------------------------------------------------------------
// kernel dispatch over compile-time shapes
// ---------------------------------------------------------------------------
template <typename TS>
void launch_setup(int G, int grid, const SetupArgs &a, hipStream_t s) {
    switch (G) {
        case 1: hipLaunchKernelGGL((k_setup<1, TS>), dim3(grid), dim3(64), 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_setup<2, TS>), dim3(grid), dim3(64), 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_setup<4, TS>), dim3(grid), dim3(64), 0, s, a); break;
        case 8: hipLaunchKernelGGL((k_setup_reg<8, TS>), dim3(grid), dim3(64), 0, s, a); break;
        case 16: hipLaunchKernelGGL((k_setup_reg<16, TS>), dim3(grid), dim3(64), 0, s, a); break;
        case 32: hipLaunchKernelGGL((k_setup_reg<32, TS>), dim3(grid), dim3(64), 0, s, a); break;
        default: hipLaunchKernelGGL((k_setup_reg<64, TS>), dim3(grid), dim3(64), 0, s, a); break;
    }
}

template <typename TS, int MODE>
void launch_apply_t(int G, int grid, const ApplyArgs &a, hipStream_t s) {
    switch (G) {
        case 1: hipLaunchKernelGGL((k_apply<1, TS, MODE>), dim3(grid), dim3(kWG), 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_apply<2, TS, MODE>), dim3(grid), dim3(kWG), 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_apply<4, TS, MODE>), dim3(grid), dim3(kWG), 0, s, a); break;
        case 8: hipLaunchKernelGGL((k_apply<8, TS, MODE>), dim3(grid), dim3(kWG), 0, s, a); break;
        case 16: hipLaunchKernelGGL((k_apply<16, TS, MODE>), dim3(grid), dim3(kWG), 0, s, a); break;
        case 32: hipLaunchKernelGGL((k_apply<32, TS, MODE>), dim3(grid), dim3(kWG), 0, s, a); break;
        default: hipLaunchKernelGGL((k_apply<64, TS, MODE>), dim3(grid), dim3(kWG), 0, s, a); break;
    }
}

template <int MODE>
void launch_apply(const bjp_precond_t *M, int grid, const ApplyArgs &a, hipStream_t s) {
    if (M->precision == BJP_FP32_STORE) launch_apply_t<float, MODE>(M->group, grid, a, s);
    else launch_apply_t<double, MODE>(M->group, grid, a, s);
}

// Launches a one-workgroup kernel with `lds` bytes of dynamic LDS (above
// 64 KB the kernel is first allowed that much).
template <typename K, typename A>
void launch_one_workgroup(K kernel, size_t lds, hipStream_t s, const A &a) {
    if (lds > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
    hipLaunchKernelGGL(kernel, dim3(1), dim3(kSmallWG), lds, s, a);
}

template <typename TS, int RES>
void launch_small_g(int G, const SmallArgs &a, size_t lds, hipStream_t s) {
    switch (G) {
        case 1: launch_one_workgroup(k_pcg_small<1, TS, true, RES>, lds, s, a); break;
        case 2: launch_one_workgroup(k_pcg_small<2, TS, true, RES>, lds, s, a); break;
        case 4: launch_one_workgroup(k_pcg_small<4, TS, true, RES>, lds, s, a); break;
        case 8: launch_one_workgroup(k_pcg_small<8, TS, true, RES>, lds, s, a); break;
        case 16: launch_one_workgroup(k_pcg_small<16, TS, true, RES>, lds, s, a); break;
        case 32: launch_one_workgroup(k_pcg_small<32, TS, true, RES>, lds, s, a); break;
        default: launch_one_workgroup(k_pcg_small<64, TS, true, RES>, lds, s, a); break;
    }
}

template <typename TS>
void launch_small_t(int G, int res, const SmallArgs &a, size_t lds, hipStream_t s) {
    switch (res) {
        case 0: launch_small_g<TS, 0>(G, a, lds, s); break;
        case kResTiles: launch_small_g<TS, kResTiles>(G, a, lds, s); break;
        case kResCsr: launch_small_g<TS, kResCsr>(G, a, lds, s); break;
        default: launch_small_g<TS, kResTiles | kResCsr>(G, a, lds, s); break;
    }
}

// What of the inverse packets and the CSR a one-workgroup kernel keeps in
// LDS beside its own `base` bytes: the packets if they fit, then the CSR if
// it fits too.
int small_residency(size_t base, int nnz, int tiles_bytes, bool has_m) {
    int res = 0;
    if (has_m && base + small_stage_bytes(kResTiles, nnz, tiles_bytes) <= kSmallLdsBytes) res |= kResTiles;
    if (base + small_stage_bytes(res | kResCsr, nnz, tiles_bytes) <= kSmallLdsBytes) res |= kResCsr;
    return res;
}

// bytes of the inverse packets (0 without a preconditioner)
int precond_tiles_bytes(const bjp_precond_t *M) {
    return M ? (int)((size_t)M->num_packets * packet_elems(M->group) *
                     (M->precision == BJP_FP32_STORE ? sizeof(float) : sizeof(double)))
             : 0;
}

// The one-workgroup solver keeps two n-vectors in LDS, then what of the
// inverse packets and the CSR fits.
void launch_small(const bjp_precond_t *M, SmallArgs a, hipStream_t s) {
    a.tiles_bytes = precond_tiles_bytes(M);
    const size_t base = 2 * sizeof(double) * (size_t)a.n;
    const int res = small_residency(base, a.nnz, a.tiles_bytes, M != nullptr);
    const size_t lds = base + small_stage_bytes(res, a.nnz, a.tiles_bytes);
    if (!M) {
        if (res & kResCsr) launch_one_workgroup(k_pcg_small<1, double, false, kResCsr>, lds, s, a);
        else launch_one_workgroup(k_pcg_small<1, double, false, 0>, lds, s, a);
    } else if (M->precision == BJP_FP32_STORE) {
        launch_small_t<float>(M->group, res, a, lds, s);
    } else {
        launch_small_t<double>(M->group, res, a, lds, s);
    }
}

// The one-workgroup Lanczos keeps two n-vectors and the step's Gram
// coefficients in LDS.
template <typename TS, int RES>
void launch_lanczos_small_g(int G, const LanczosSmallArgs &a, size_t lds, hipStream_t s) {
    switch (G) {
        case 1: launch_one_workgroup(k_lanczos_small<1, TS, true, RES>, lds, s, a); break;
        case 2: launch_one_workgroup(k_lanczos_small<2, TS, true, RES>, lds, s, a); break;
        case 4: launch_one_workgroup(k_lanczos_small<4, TS, true, RES>, lds, s, a); break;
        case 8: launch_one_workgroup(k_lanczos_small<8, TS, true, RES>, lds, s, a); break;
        case 16: launch_one_workgroup(k_lanczos_small<16, TS, true, RES>, lds, s, a); break;
        case 32: launch_one_workgroup(k_lanczos_small<32, TS, true, RES>, lds, s, a); break;
        default: launch_one_workgroup(k_lanczos_small<64, TS, true, RES>, lds, s, a); break;
    }
}

template <typename TS>
void launch_lanczos_small_t(int G, int res, const LanczosSmallArgs &a, size_t lds, hipStream_t s) {
    switch (res) {
        case 0: launch_lanczos_small_g<TS, 0>(G, a, lds, s); break;
        case kResTiles: launch_lanczos_small_g<TS, kResTiles>(G, a, lds, s); break;
        case kResCsr: launch_lanczos_small_g<TS, kResCsr>(G, a, lds, s); break;
        default: launch_lanczos_small_g<TS, kResTiles | kResCsr>(G, a, lds, s); break;
    }
}

// The one-workgroup estimate keeps two n-vectors and the coefficients in
// LDS, then what of the inverse packets and the CSR fits (small_residency).
void launch_lanczos_small(const bjp_precond_t *M, LanczosSmallArgs a, hipStream_t s) {
    a.tiles_bytes = precond_tiles_bytes(M);
    const size_t base = sizeof(double) * (2 * (size_t)a.n + lanczos_coef_slots(a.steps));
    const int res = small_residency(base, a.nnz, a.tiles_bytes, M != nullptr);
    const size_t lds = base + small_stage_bytes(res, a.nnz, a.tiles_bytes);
    if (!M) {
        if (res & kResCsr) launch_one_workgroup(k_lanczos_small<1, double, false, kResCsr>, lds, s, a);
        else launch_one_workgroup(k_lanczos_small<1, double, false, 0>, lds, s, a);
    } else if (M->precision == BJP_FP32_STORE) {
        launch_lanczos_small_t<float>(M->group, res, a, lds, s);
    } else {
        launch_lanczos_small_t<double>(M->group, res, a, lds, s);
    }
}

// gs = lanes per row of the lane-group schedule; 0 = row-block streaming with
// stages of 4 entries per thread, kStream7 = with stages of 7.
constexpr int kStream7 = -7;
template <int MODE>
void launch_spmv(int gs, int grid, const SpmvArgs &a, hipStream_t s) {
    switch (gs) {
        case 0: hipLaunchKernelGGL((k_spmv_stream<MODE, 4>), dim3(grid), dim3(kWG), 0, s, a); break;
        case kStream7: hipLaunchKernelGGL((k_spmv_stream<MODE, 7>), dim3(grid), dim3(kWG), 0, s, a); break;
        case 1: hipLaunchKernelGGL((k_spmv<1, MODE>), dim3(grid), dim3(kWG), 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_spmv<2, MODE>), dim3(grid), dim3(kWG), 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_spmv<4, MODE>), dim3(grid), dim3(kWG), 0, s, a); break;
        case 8: hipLaunchKernelGGL((k_spmv<8, MODE>), dim3(grid), dim3(kWG), 0, s, a); break;
        case 16: hipLaunchKernelGGL((k_spmv<16, MODE>), dim3(grid), dim3(kWG), 0, s, a); break;
        case 32: hipLaunchKernelGGL((k_spmv<32, MODE>), dim3(grid), dim3(kWG), 0, s, a); break;
        default: hipLaunchKernelGGL((k_spmv<64, MODE>), dim3(grid), dim3(kWG), 0, s, a); break;
    }
}

// Launch shape of the row-streaming kernels.
struct RowLaunch {
    int grid, chunk;
};

RowLaunch spmv_shape(int n, int gs) {
    if (gs <= 0) {
        // whole row blocks per workgroup
        const int blocks = ceil_div(std::max(n, 1), kStreamRows);
        const int per = ceil_div(blocks, kMaxRedWG);
        const int chunk = per * kStreamRows;
        return {round8(ceil_div(std::max(n, 1), chunk)), chunk};
    }
    const int u = spmv_rows_per_group(gs);
    const int rows_per_step = (kWG / gs) * u;
    const int grid = round8(std::min(ceil_div(n, rows_per_step), kMaxRedWG));
    return {grid, ceil_div(n, grid)};
}

// Compute units of the current device (cached per device).
int device_cus() {
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cus[dev] = v;
    }
    return cus[dev];
}

// The block-inverse application runs one workgroup per compute unit for
// 64-row groups: each wave streams a long sequence of packets (every W-th
// packet, W waves in the launch) through its two-stage pipeline, which keeps
// more bytes in flight than more, shorter-lived waves (measured at 128^3,
// n_b = 64: 117 us at 256 workgroups, 120 at 512, 127 at 768; FP32 tiles:
// 49.7 us at one workgroup per CU, 51.0 at two).  Narrower groups have
// smaller packets, and one workgroup per CU then holds too few bytes in
// flight to cover the memory latency: those launches take enough workgroups
// per CU to keep about 16 KB of packets (tiles and vectors) in their
// pipelines per CU (measured at 128^3: n_b = 8 24.0 -> 18.9 us, n_b = 32 FP32
// 38.7 -> 30.7 us; 32 KB per CU was slower for every block size).
constexpr int kApplyInflight = 16384;

RowLaunch apply_shape(const bjp_precond_t *M) {
    const int packets = M->num_packets;
    const int elem = M->precision == BJP_FP32_STORE ? 4 : 8;
    const int bytes = M->packet_elems * elem + 64 * 32;   // tiles + q, r read, r, z written
    const int per_cu = M->group == 64 ? 1 : std::max(1, std::min(8, (kApplyInflight + bytes - 1) / bytes));
    const int grid = round8(std::min(ceil_div(packets, kWaves), std::min(device_cus() * per_cu, kMaxRedWG)));
    return {grid, ceil_div(packets, grid)};
}

RowLaunch rows_shape(int n) {
    const int grid = round8(std::min(ceil_div(n, kWG), kMaxRedWG));
    return {grid, ceil_div(n, grid)};
}

RowLaunch gram_shape(int n) {
    const int per = kWG * kGramRows;
    const int grid = round8(ceil_div(n, per));
    return {grid, per};
}

// A handle must describe a partition whose packets the kernels can address.
bool precond_ok(const bjp_precond_t *M, int n) {
    if (!M || M->n != n || !M->tiles || !M->offsets) return false;
    const int G = M->group;
    if (G < 1 || G > 64 || (G & (G - 1))) return false;
    if (M->num_blocks < (n > 0 ? 1 : 0) || M->num_packets != ceil_div(M->num_blocks, 64 / G)) return false;
    if (M->packet_elems != packet_elems(G)) return false;
    if (M->precision != BJP_FP64 && M->precision != BJP_FP32_STORE) return false;
    if (M->block_size < 0 || M->block_size > G) return false;
    if (M->block_size > 0 && M->num_blocks != ceil_div(n, M->block_size)) return false;
    return true;
}

// Lanes per CSR row: the largest power of two not above the mean row length
// (measured on the 7-point stencil: 4 lanes beat 8 and 16).
int auto_lanes(const bjp_csr_t *A) {
    if (A->n <= 0) return 4;
    const double mean = (double)A->nnz / A->n;
    int gs = 1;
    while (gs < 64 && 2 * gs <= mean) gs <<= 1;
    return gs;
}

#ifndef BJP_STREAM_MEAN
#define BJP_STREAM_MEAN 12.0
#endif
// Schedule of the single-system products: row-block streaming (0) for short
// rows, else the lane-group schedule with auto_lanes lanes.
// Streaming stage size from the mean row length.
int stream_schedule(const bjp_csr_t *A) {
    return A->n > 0 && (double)A->nnz <= 7.0 * A->n ? kStream7 : 0;
}
int auto_spmv(const bjp_csr_t *A) {
    if (A->n > 0 && (double)A->nnz / A->n < BJP_STREAM_MEAN) return stream_schedule(A);
    return auto_lanes(A);
}

// Schedule from the user's option: > 0 lanes per row, < 0 streaming, 0 auto.
int spmv_schedule(int opt, const bjp_csr_t *A) {
    if (opt > 0) return pow2_at_least(std::min(opt, 64));
    if (opt < 0) return stream_schedule(A);
    return auto_spmv(A);
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
// Owner of the batch solver's captured graph and capture stream.
struct GraphGuard {
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    GraphGuard() = default;
    GraphGuard(const GraphGuard &) = delete;
    GraphGuard &operator=(const GraphGuard &) = delete;
    ~GraphGuard() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (cap) (void)hipStreamDestroy(cap);
    }
};
struct BatchPlan {
    std::vector<SysInfo> sys;
    std::vector<int32_t> off;        // per system: nblocks+1 global row offsets
    std::vector<long long> off_base; // index of each system's first offset
    std::vector<int> block_base;     // global index of each system's first block
    size_t tile_scalars = 0;
};

int make_batch_plan(const bjp_csr_t *A, const bjp_batch_t *B, BatchPlan &P) {
    if (!B || B->num_systems <= 0 || !B->sys_rows || !B->block_size) return BJP_EINVAL;
    const int S = B->num_systems;
    if (B->sys_rows[0] != 0 || B->sys_rows[S] != A->n) return BJP_EINVAL;
    P.sys.resize(S);
    P.off.clear();
    P.off_base.resize(S);
    P.block_base.resize(S);
    long long tiles = 0;
    int blocks = 0;
    for (int s = 0; s < S; ++s) {
        const int r0 = B->sys_rows[s], r1 = B->sys_rows[s + 1], nb = B->block_size[s];
        if (r1 <= r0 || nb < 1 || nb > BJP_MAX_BLOCK) return BJP_EINVAL;
        SysInfo &si = P.sys[s];
        si.row0 = r0;
        si.n = r1 - r0;
        si.nb = nb;
        si.G = pow2_at_least(std::min(nb, si.n));
        si.nblocks = ceil_div(si.n, nb);
        si.packets = ceil_div(si.nblocks, 64 / si.G);
        si.tile0 = tiles;
        tiles += (long long)si.packets * packet_elems(si.G);
        P.off_base[s] = (long long)P.off.size();
        P.block_base[s] = blocks;
        blocks += si.nblocks;
        for (long long r = r0; r < r1; r += nb) P.off.push_back((int32_t)r);
        P.off.push_back(r1);
    }
    P.tile_scalars = (size_t)tiles;
    return BJP_OK;
}

size_t batch_precond_bytes(const BatchPlan &P, int precision) {
    const size_t elem = precision == BJP_FP32_STORE ? 4 : 8;
    return al256(sizeof(SysInfo) * P.sys.size()) + al256(sizeof(int32_t) * (P.sys.size() + 1)) +
           al256(sizeof(int32_t) * P.off.size()) + al256(P.tile_scalars * elem) + al256(64) +
           al256(sizeof(SetupSys) * P.sys.size());
}

template <typename TS>
void launch_setup_batch(int G, int grid, const SetupArgs &a, const SetupSys *items, int count, hipStream_t s) {
    switch (G) {
        case 1: hipLaunchKernelGGL((k_setup_batch<1, TS>), dim3(grid), dim3(64), 0, s, a, items, count); break;
        case 2: hipLaunchKernelGGL((k_setup_batch<2, TS>), dim3(grid), dim3(64), 0, s, a, items, count); break;
        case 4: hipLaunchKernelGGL((k_setup_batch<4, TS>), dim3(grid), dim3(64), 0, s, a, items, count); break;
        case 8: hipLaunchKernelGGL((k_setup_batch<8, TS>), dim3(grid), dim3(64), 0, s, a, items, count); break;
        case 16: hipLaunchKernelGGL((k_setup_batch<16, TS>), dim3(grid), dim3(64), 0, s, a, items, count); break;
        case 32: hipLaunchKernelGGL((k_setup_batch<32, TS>), dim3(grid), dim3(64), 0, s, a, items, count); break;
        default: hipLaunchKernelGGL((k_setup_batch<64, TS>), dim3(grid), dim3(64), 0, s, a, items, count); break;
    }
}

// Packets per apply tile of the batched solver (16 per wave: the two-stage
// pipeline runs long enough to pay for its start; measured on the 512-system
// batch: 55.1 ms per solve at 16 packets per tile, 54.7 at 32, 54.3 at 64).
constexpr int kPacketsPerTile = 64;

struct BatchTables {
    std::vector<Tile> rt, pt;               // row tiles (grouped by SpMV schedule), packet tiles (by G)
    std::vector<int> rt_begin, rt_end;      // per system
    std::vector<int> pt_begin, pt_end;      // per system
    std::vector<int> rs_gs, rs_begin, rs_end;    // row-tile range of each SpMV schedule
    std::vector<int> cls_g, cls_begin, cls_end;  // packet-tile range of each width G
};

// Row tiles of sys_tile_rows[s] rows per system, grouped by the system's SpMV
// schedule sys_gs[s] (one product launch per schedule present; a system's
// tiles stay contiguous); packet tiles grouped by lane-group width.
void make_batch_tables(const BatchPlan &P, const std::vector<int> &sys_tile_rows, const std::vector<int> &sys_gs,
                       BatchTables &T) {
    const int S = (int)P.sys.size();
    T.rt_begin.assign(S, 0);
    T.rt_end.assign(S, 0);
    T.pt_begin.assign(S, 0);
    T.pt_end.assign(S, 0);
    std::vector<int> kinds(sys_gs);
    std::sort(kinds.begin(), kinds.end());
    kinds.erase(std::unique(kinds.begin(), kinds.end()), kinds.end());
    for (const int g : kinds) {
        const int b = (int)T.rt.size();
        for (int s = 0; s < S; ++s) {
            if (sys_gs[s] != g) continue;
            const SysInfo &si = P.sys[s];
            const int tr = sys_tile_rows[s];
            T.rt_begin[s] = (int)T.rt.size();
            for (int r = si.row0; r < si.row0 + si.n; r += tr)
                T.rt.push_back(Tile{s, r, std::min(r + tr, si.row0 + si.n), 0});
            T.rt_end[s] = (int)T.rt.size();
        }
        if ((int)T.rt.size() > b) {
            T.rs_gs.push_back(g);
            T.rs_begin.push_back(b);
            T.rs_end.push_back((int)T.rt.size());
        }
    }
    for (int G = 1; G <= 64; G <<= 1) {
        const int b = (int)T.pt.size();
        for (int s = 0; s < S; ++s) {
            const SysInfo &si = P.sys[s];
            if (si.G != G) continue;
            T.pt_begin[s] = (int)T.pt.size();
            for (int pk = 0; pk < si.packets; pk += kPacketsPerTile)
                T.pt.push_back(Tile{s, pk, std::min(pk + kPacketsPerTile, si.packets), 0});
            T.pt_end[s] = (int)T.pt.size();
        }
        if ((int)T.pt.size() > b) {
            T.cls_g.push_back(G);
            T.cls_begin.push_back(b);
            T.cls_end.push_back((int)T.pt.size());
        }
    }
}

size_t batch_tiles_bound(const BatchPlan &P, int min_tile_rows, size_t *nrt, size_t *npt) {
    size_t r = 0, p = 0;
    for (const SysInfo &si : P.sys) {
        r += (size_t)ceil_div(si.n, min_tile_rows);
        p += (size_t)ceil_div(si.packets, kPacketsPerTile);
    }
    *nrt = r;
    *npt = p;
    return r + p;
}

template <int MODE>
void launch_spmv_tiles(int gs, int grid, const SpmvArgs &a, const TileSpan &t, hipStream_t s) {
    switch (gs) {
        case 0:
        case kStream7: hipLaunchKernelGGL((k_spmv_tiles_stream<MODE>), dim3(grid), dim3(kWG), 0, s, a, t); break;
        case 1: hipLaunchKernelGGL((k_spmv_tiles<1, MODE>), dim3(grid), dim3(kWG), 0, s, a, t); break;
        case 2: hipLaunchKernelGGL((k_spmv_tiles<2, MODE>), dim3(grid), dim3(kWG), 0, s, a, t); break;
        case 4: hipLaunchKernelGGL((k_spmv_tiles<4, MODE>), dim3(grid), dim3(kWG), 0, s, a, t); break;
        case 8: hipLaunchKernelGGL((k_spmv_tiles<8, MODE>), dim3(grid), dim3(kWG), 0, s, a, t); break;
        case 16: hipLaunchKernelGGL((k_spmv_tiles<16, MODE>), dim3(grid), dim3(kWG), 0, s, a, t); break;
        case 32: hipLaunchKernelGGL((k_spmv_tiles<32, MODE>), dim3(grid), dim3(kWG), 0, s, a, t); break;
        default: hipLaunchKernelGGL((k_spmv_tiles<64, MODE>), dim3(grid), dim3(kWG), 0, s, a, t); break;
    }
}

template <typename TS, int MODE>
void launch_apply_tiles_t(int G, int grid, const ApplyArgs &a, const TileSpan &t, hipStream_t s) {
    switch (G) {
        case 1: hipLaunchKernelGGL((k_apply_tiles<1, TS, MODE>), dim3(grid), dim3(kWG), 0, s, a, t); break;
        case 2: hipLaunchKernelGGL((k_apply_tiles<2, TS, MODE>), dim3(grid), dim3(kWG), 0, s, a, t); break;
        case 4: hipLaunchKernelGGL((k_apply_tiles<4, TS, MODE>), dim3(grid), dim3(kWG), 0, s, a, t); break;
        case 8: hipLaunchKernelGGL((k_apply_tiles<8, TS, MODE>), dim3(grid), dim3(kWG), 0, s, a, t); break;
        case 16: hipLaunchKernelGGL((k_apply_tiles<16, TS, MODE>), dim3(grid), dim3(kWG), 0, s, a, t); break;
        case 32: hipLaunchKernelGGL((k_apply_tiles<32, TS, MODE>), dim3(grid), dim3(kWG), 0, s, a, t); break;
        default: hipLaunchKernelGGL((k_apply_tiles<64, TS, MODE>), dim3(grid), dim3(kWG), 0, s, a, t); break;
    }
}

// Two pinned host slots per host thread for the solver's overlapped polls
// (allocated on first use, kept for the life of the thread's process).
PcgState *pinned_states() {
    static thread_local PcgState *p = nullptr;
    if (!p) {
        void *q = nullptr;
        if (hipHostMalloc(&q, 2 * sizeof(PcgState), hipHostMallocDefault) != hipSuccess) return nullptr;
        p = static_cast<PcgState *>(q);
    }
    return p;
}

struct EventPair {
    hipEvent_t e[2] = {nullptr, nullptr};
    EventPair() = default;
    EventPair(const EventPair &) = delete;
    EventPair &operator=(const EventPair &) = delete;
    ~EventPair() {
        for (hipEvent_t v : e)
            if (v) (void)hipEventDestroy(v);
    }
};

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *bjp_status_string(int status) {
    switch (status) {
        case BJP_OK: return "BJP_OK";
        case BJP_EINVAL: return "BJP_EINVAL";
        case BJP_ENOTSPD: return "BJP_ENOTSPD";
        case BJP_ENOCONV: return "BJP_ENOCONV";
        case BJP_EBREAKDOWN: return "BJP_EBREAKDOWN";
        case BJP_ENONFINITE: return "BJP_ENONFINITE";
        case BJP_EWORKSPACE: return "BJP_EWORKSPACE";
        case BJP_EHIP: return "BJP_EHIP";
        default: return "BJP_UNKNOWN";
    }
}

int bjp_precondition_workspace(const bjp_csr_t *A, const bjp_block_spec_t *spec, int precision,
                               size_t *bytes) {
    if (!bytes) return BJP_EINVAL;
    *bytes = 0;
    if (check_csr_host(A) != BJP_OK) return BJP_EINVAL;
    if (precision != BJP_FP64 && precision != BJP_FP32_STORE) return BJP_EINVAL;
    Partition P;
    const int st = make_partition(A->n, spec, P);
    if (st != BJP_OK) return st;
    *bytes = precond_ws_bytes(P, precision);
    return BJP_OK;
}

int bjp_precondition(const bjp_csr_t *A, const bjp_block_spec_t *spec, int precision, void *ws,
                     size_t ws_bytes, bjp_precond_t *M_out, int32_t *failed_block, hipStream_t stream) {
    if (failed_block) *failed_block = -1;
    if (!M_out) return BJP_EINVAL;
    std::memset(M_out, 0, sizeof(*M_out));
    if (check_csr_host(A) != BJP_OK) return BJP_EINVAL;
    if (precision != BJP_FP64 && precision != BJP_FP32_STORE) return BJP_EINVAL;
    Partition P;
    int st = make_partition(A->n, spec, P);
    if (st != BJP_OK) return st;
    const size_t need = precond_ws_bytes(P, precision);
    if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255)) return BJP_EWORKSPACE;

    Carver cv{static_cast<char *>(ws)};
    int32_t *off = cv.take<int32_t>((size_t)P.nblocks + 1);
    void *tiles = cv.base + cv.used;
    cv.used += al256((size_t)P.packets * P.E * (precision == BJP_FP32_STORE ? 4 : 8));
    int32_t *flags = cv.take<int32_t>(16);

    M_out->n = A->n;
    M_out->block_size = P.uniform;
    M_out->num_blocks = P.nblocks;
    M_out->precision = precision;
    M_out->group = P.G;
    M_out->num_packets = P.packets;
    M_out->packet_elems = P.E;
    M_out->offsets = off;
    M_out->tiles = tiles;

    st = run_validate(A, flags, stream);
    if (st != BJP_OK) return st;
    if (P.uniform > 0)
        hipLaunchKernelGGL(k_uniform_offsets, dim3(std::min(ceil_div(P.nblocks + 1, kWG), 4096)), dim3(kWG), 0,
                           stream, off, P.nblocks, P.uniform, A->n);
    else
        HIP_TRY(hipMemcpyAsync(off, P.off.data(), sizeof(int32_t) * P.off.size(), hipMemcpyHostToDevice,
                               stream));
    if (A->n == 0) {
        HIP_TRY(hipStreamSynchronize(stream));
        return BJP_OK;
    }
    SetupArgs sa{A->row_ptr, A->col_idx, A->val, off, P.nblocks, tiles, flags, 0};
    if (precision == BJP_FP32_STORE) launch_setup<float>(P.G, P.packets, sa, stream);
    else launch_setup<double>(P.G, P.packets, sa, stream);
    HIP_TRY(hipGetLastError());
    int32_t h[4];
    HIP_TRY(hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (h[0] != INT_MAX) {
        if (failed_block) *failed_block = h[0];
        return BJP_ENOTSPD;
    }
    return BJP_OK;
}

int bjp_apply(const bjp_precond_t *M, const double *r, double *z, hipStream_t stream) {
    if (!M || M->n < 0) return BJP_EINVAL;
    if (M->n == 0) return BJP_OK;
    if (!r || !z || !precond_ok(M, M->n)) return BJP_EINVAL;
    ApplyArgs a{};
    a.nblocks = M->num_blocks;
    a.num_packets = M->num_packets;
    a.n = M->n;
    a.uniform_nb = M->block_size;
    a.off = M->offsets;
    a.tiles = M->tiles;
    a.rin = r;
    a.zout = z;
    const RowLaunch L = apply_shape(M);
    launch_apply<APPLY_PLAIN>(M, L.grid, a, stream);
    HIP_TRY(hipGetLastError());
    return BJP_OK;
}

}  // extern "C"

namespace {

// Column panels (see spmv.hpp) need rows of at least kPanelMeanRow entries
// on average; they are chosen automatically once the gathered vector is
// larger than an XCD's L2 could hold (n >= 2^20 rows, 8 MB), or forced with
// spmv_lanes = -2.
constexpr int kPanelMeanRow = 12;
bool panels_possible(const bjp_csr_t *A) {
    return A->n >= kPanels * 64 && (double)A->nnz >= (double)kPanelMeanRow * A->n;
}
bool use_panels(int opt, const bjp_csr_t *A) {
    if (opt == -2) return panels_possible(A);
    return opt == 0 && panels_possible(A) && A->n >= (1 << 20);
}
int panel_nscan(int n) { return ceil_div(std::max(n, 1), kScanRows); }
// Panel-major copy of A, its row pointers and the partial products (the
// per-(panel, row) counts of the build share the partial products' space).
size_t panel_bytes(const bjp_csr_t *A) {
    if (!panels_possible(A)) return 0;
    const size_t n = (size_t)A->n, nnz = (size_t)A->nnz;
    return al256(sizeof(int32_t) * kPanels * (size_t)panel_nscan(A->n)) + al256(sizeof(int32_t) * kPanels * (n + 1)) +
           al256(sizeof(int32_t) * nnz) + al256(sizeof(double) * nnz) + al256(sizeof(double) * kPanels * n);
}

// Short rows (the automatic streaming regime) get 16-bit column offsets.
bool short_rows(const bjp_csr_t *A) { return A->n > 0 && (double)A->nnz / A->n < BJP_STREAM_MEAN; }
size_t delta16_bytes(const bjp_csr_t *A) {
    return short_rows(A) ? al256(sizeof(int16_t) * (size_t)std::max(A->nnz, 1)) + al256(64) : 0;
}

// PCG workspace: five vectors, two sets of reduction partials, two states,
// flags, zeros, the 16-bit column offsets (short rows) and, when allowed,
// the column-panel copy (long rows).
size_t pcg_ws_bytes(const bjp_csr_t *A, bool with_panels) {
    const size_t vec = al256(sizeof(double) * (size_t)std::max(A->n, 1));
    return 5 * vec + 2 * al256(sizeof(double) * 2 * kMaxRedWG) + 2 * al256(sizeof(PcgState)) + 2 * al256(64) +
           (with_panels ? panel_bytes(A) : 0) + delta16_bytes(A);
}

}  // namespace

extern "C" {

int bjp_pcg_workspace(const bjp_csr_t *A, size_t *bytes) {
    if (!bytes) return BJP_EINVAL;
    *bytes = 0;
    if (check_csr_host(A) != BJP_OK) return BJP_EINVAL;
    *bytes = pcg_ws_bytes(A, true);
    return BJP_OK;
}

}  // extern "C"

namespace {

// The solver behind bjp_pcg_solve and bjp_pcg_solve_noalloc.  no_alloc: the
// workspace is the library's static scratch and nothing may be allocated, so
// the iteration's product never takes the column panels (their copy of A is
// not part of the scratch) and the host polls read the state into ordinary
// host memory with a stream synchronisation (no pinned slots, no events).
int pcg_solve_impl(const bjp_csr_t *A, const bjp_precond_t *M, const double *b, double *x,
                   const bjp_pcg_opts_t *opts, void *ws, size_t ws_bytes, bjp_pcg_info_t *info,
                   hipStream_t stream, bool no_alloc) {
    if (!info) return BJP_EINVAL;
    std::memset(info, 0, sizeof(*info));
    auto fail = [&](int st) {
        info->status = st;
        return st;
    };
    if (check_csr_host(A) != BJP_OK) return fail(BJP_EINVAL);
    const int n = A->n;
    if (n > 0 && (!b || !x)) return fail(BJP_EINVAL);
    if (M && n > 0 && !precond_ok(M, n)) return fail(BJP_EINVAL);
    bjp_pcg_opts_t o{};
    if (opts) o = *opts;
    if (!(o.tol > 0.0)) o.tol = 1e-10;
    if (o.max_iter <= 0) o.max_iter = std::max(n, 1);
    if (o.max_replacements == 0) o.max_replacements = 3;
    else if (o.max_replacements < 0) o.max_replacements = 0;
    if (o.check_every <= 0) o.check_every = 16;
    if (no_alloc && o.spmv_lanes == -2) return fail(BJP_EINVAL);
    const size_t need = pcg_ws_bytes(A, !no_alloc);
    if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255)) return fail(BJP_EWORKSPACE);
    if (n == 0) return fail(BJP_OK);

    Carver cv{static_cast<char *>(ws)};
    double *r = cv.take<double>(n), *z = cv.take<double>(n), *p0 = cv.take<double>(n);
    double *p1 = cv.take<double>(n), *q = cv.take<double>(n);
    // partials of the products (p^T A p, residual norms) and of the
    // preconditioner applications (r^T z, r^T r) are kept apart: each
    // streaming launch reads the other's as the input of its decision
    double *partials = cv.take<double>(2 * kMaxRedWG);
    double *partials_a = cv.take<double>(2 * kMaxRedWG);
    // st: the state between iterations (after the application); st1: after
    // the direction update.  Each iteration's two deciding launches read one
    // and record the other.
    PcgState *st = cv.take<PcgState>(1);
    PcgState *st1 = cv.take<PcgState>(1);
    int32_t *flags = cv.take<int32_t>(16);
    double *zeros = cv.take<double>(8);
    if (!M) z = r;  // plain CG: the "preconditioned" residual is r itself

    int s = run_validate(A, flags, stream);
    if (s != BJP_OK) return fail(s);

    // Small systems (automatic product schedule, no kernel timing): the whole
    // solve in one workgroup (small.hpp), the same algorithm and decisions.
    if (n <= kSmallMaxRows && (long long)A->nnz <= (long long)kSmallMaxMeanRow * n && o.spmv_lanes == 0 &&
        !o.timing) {
        SmallArgs sm{};
        sm.n = n;
        sm.nnz = (int)A->nnz;
        sm.rp = A->row_ptr;
        sm.ci = A->col_idx;
        sm.val = A->val;
        sm.b = b;
        sm.x = x;
        if (M) {
            sm.nblocks = M->num_blocks;
            sm.num_packets = M->num_packets;
            sm.uniform_nb = M->block_size;
            sm.off = M->offsets;
            sm.tiles = M->tiles;
        }
        sm.tol = o.tol;
        sm.max_iter = o.max_iter;
        sm.max_repl = o.max_replacements;
        sm.x0_given = o.x0_given;
        sm.hist = o.history;
        sm.out = st;
        sm.repl_out = flags + 8;
        launch_small(M, sm, stream);
        HIP_TRY(hipGetLastError());
        PcgState h{};
        int32_t rep = 0;
        HIP_TRY(hipMemcpyAsync(&h, st, sizeof(PcgState), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipMemcpyAsync(&rep, flags + 8, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        info->status = h.status;
        info->iterations = h.it;
        info->replacements = rep;
        info->polls = 1;
        info->rel_res_recursive = h.relres;
        info->rel_res_true = h.relres_true;
        return h.status;
    }

    // the iteration's product q = A p: column panels or the CSR schedule;
    // the residual products always take the CSR schedule
    const bool panels = !no_alloc && use_panels(o.spmv_lanes, A);
    if (o.spmv_lanes == -2 && !panels) return fail(BJP_EINVAL);
    const int gs = spmv_schedule(o.spmv_lanes == -2 ? 0 : o.spmv_lanes, A);
    const RowLaunch Ls = spmv_shape(n, gs);
    PanelArgs pa{};
    const RowLaunch Lf = rows_shape(n);
    const int panel_grid = kPanels * std::min(ceil_div(n, kPanelChunk), 8 * device_cus() / kPanels * 4);
    if (panels) {
        pa.n = n;
        pa.nnz = A->nnz;
        pa.width = ceil_div(n, kPanels);
        pa.rp = A->row_ptr;
        pa.ci = A->col_idx;
        pa.val = A->val;
        pa.nscan = panel_nscan(n);
        pa.bsum = cv.take<int32_t>((size_t)kPanels * pa.nscan);
        pa.prp = cv.take<int32_t>((size_t)kPanels * ((size_t)n + 1));
        pa.pci = cv.take<int32_t>((size_t)A->nnz);
        pa.pval = cv.take<double>((size_t)A->nnz);
        pa.Y = cv.take<double>((size_t)kPanels * n);
        pa.cnt = reinterpret_cast<int32_t *>(pa.Y);
        const int rgrid = std::min(ceil_div(n, kWG / kBuildLanes), 8192);
        hipLaunchKernelGGL(k_panel_count, dim3(rgrid), dim3(kWG), 0, stream, pa);
        hipLaunchKernelGGL(k_panel_blocksum, dim3(pa.nscan), dim3(kWG), 0, stream, pa);
        hipLaunchKernelGGL(k_panel_blockscan, dim3(1), dim3(kWG), 0, stream, pa);
        hipLaunchKernelGGL(k_panel_offsets, dim3(pa.nscan), dim3(kWG), 0, stream, pa);
        hipLaunchKernelGGL(k_panel_scatter, dim3(rgrid), dim3(kWG), 0, stream, pa);
        HIP_TRY(hipGetLastError());
    }
    // the iteration's streaming product reads 16-bit column offsets when
    // they all fit (decided on the device)
    const int16_t *cd = nullptr;
    int32_t *cd_bad = nullptr;
    if (short_rows(A)) {
        int16_t *cdw = cv.take<int16_t>((size_t)std::max(A->nnz, 1));
        cd_bad = cv.take<int32_t>(16);
        if (!panels && gs <= 0 && A->nnz > 0) {
            hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, stream, cd_bad, 1, 0);
            hipLaunchKernelGGL(k_col_delta16, dim3(std::min(ceil_div(n, kWG), 4096)), dim3(kWG), 0, stream,
                               A->row_ptr, A->col_idx, n, cdw, cd_bad);
            cd = cdw;
        }
    }
    const RowLaunch La = M ? apply_shape(M) : rows_shape(n);
    const int fill_grid = std::min(ceil_div(n, kWG), 4096);

    hipLaunchKernelGGL(k_pcg_state_init, dim3(1), dim3(64), 0, stream, st, o.tol, o.max_iter);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, stream, zeros, 8, 0.0);
    hipLaunchKernelGGL(k_fill, dim3(fill_grid), dim3(kWG), 0, stream, p0, n, 0.0);
    hipLaunchKernelGGL(k_fill, dim3(fill_grid), dim3(kWG), 0, stream, p1, n, 0.0);
    if (!o.x0_given) hipLaunchKernelGGL(k_fill, dim3(fill_grid), dim3(kWG), 0, stream, x, n, 0.0);

    SpmvArgs sa{};
    sa.n = n;
    sa.chunk = Ls.chunk;
    sa.rp = A->row_ptr;
    sa.ci = A->nnz > 0 ? A->col_idx : reinterpret_cast<const int32_t *>(zeros);
    sa.val = A->nnz > 0 ? A->val : zeros;
    sa.st = st;
    sa.p0 = p0;
    sa.p1 = p1;
    sa.q = q;
    sa.b = b;
    sa.x = x;
    sa.r = r;
    sa.partials = partials;

    FinishArgs fa{};
    fa.st = st;
    fa.partials = partials;
    fa.hist = o.history;

    ApplyArgs aa{};
    aa.n = n;
    if (M) {
        aa.nblocks = M->num_blocks;
        aa.num_packets = M->num_packets;
        aa.uniform_nb = M->block_size;
        aa.off = M->offsets;
        aa.tiles = M->tiles;
    }
    aa.rin = r;
    aa.zout = z;
    aa.st = st;
    aa.x = x;
    aa.r = r;
    aa.q = q;
    aa.p0 = p0;
    aa.p1 = p1;
    aa.partials = partials_a;
    // the iteration's application reads st1 and the product's partials
    ApplyArgs au = aa;
    au.st = st1;
    au.st_out = st;
    au.dec_partials = partials;
    au.dec_nparts = panels ? Lf.grid : Ls.grid;
    SpmvArgs su = sa;
    su.st = st1;
    su.cd = cd;
    su.cd_bad = cd_bad;
    SpmvArgs suf = su;      // the panel launches' row finish
    suf.chunk = Lf.chunk;
    FinishArgs fu = fa;
    fu.partials = partials_a;

    auto start_direction = [&]() {
        if (M) launch_apply<APPLY_INIT>(M, La.grid, aa, stream);
        else hipLaunchKernelGGL((k_rows_update<APPLY_INIT>), dim3(La.grid), dim3(kWG), 0, stream, aa, n,
                                La.chunk);
        finish<FIN_PCG_START>(fu, La.grid, stream);
    };
    bjp_timing_t *tm = o.timing;
    if (tm) tm->recorded = 0;
    const int tm_stride = tm && tm->stride > 1 ? tm->stride : 1;
    long long tm_seen = 0;      // launches of the timed kernel so far
    auto mark = [&](int kernel, int which) {
        if (!tm || tm->kernel != kernel || !tm->events) return;
        const bool timed = tm_seen % tm_stride == 0 && tm->recorded < tm->capacity;
        if (timed) (void)hipEventRecord(tm->events[2 * tm->recorded + which], stream);
        if (which == 1) {
            if (timed) tm->recorded++;
            ++tm_seen;
        }
    };
    // One iteration is three launches, each taking the scalar decision of the
    // previous one as its prologue (no separate finish launches):
    //   direction     update decision (rho, beta, convergence) -> st1;
    //                 x += alpha p (owed by the last step); p = z + beta p
    //   product       q = A p, partials of p^T q
    //   application   alpha = rho / p^T q -> st; r -= alpha q, z = M^-1 r,
    //                 partials of r^T z, r^T r (decision pending, x update owed)
    // Moving x += alpha p to the direction update, which reads p anyway, saves
    // one vector pass per iteration.
    const int dir_grid = std::min(ceil_div(n, kWG * kDirRows), 2048);
    auto iteration = [&]() {
        if (M)
            hipLaunchKernelGGL((k_direction<FIN_PCG_UPDATE>), dim3(dir_grid), dim3(kWG), 0, stream, st, st1,
                               partials_a, La.grid, o.history, z, p0, p1, x, n);
        else
            hipLaunchKernelGGL((k_direction<FIN_PCG_UPDATE_I>), dim3(dir_grid), dim3(kWG), 0, stream, st, st1,
                               partials_a, La.grid, o.history, z, p0, p1, x, n);
        mark(BJP_KERNEL_SPMV, 0);
        if (panels) {
            hipLaunchKernelGGL(k_spmv_panels<SPMV_SIGMA>, dim3(panel_grid), dim3(kWG), 0, stream, su, pa);
            hipLaunchKernelGGL(k_panel_finish<SPMV_SIGMA>, dim3(Lf.grid), dim3(kWG), 0, stream, suf, pa);
        } else {
            launch_spmv<SPMV_SIGMA>(gs, Ls.grid, su, stream);
        }
        mark(BJP_KERNEL_SPMV, 1);
        mark(BJP_KERNEL_APPLY, 0);
        if (M) launch_apply<APPLY_STEP>(M, La.grid, au, stream);
        else hipLaunchKernelGGL((k_rows_update<APPLY_STEP>), dim3(La.grid), dim3(kWG), 0, stream, au,
                                n, La.chunk);
        mark(BJP_KERNEL_APPLY, 1);
    };
    // the x update still owed when the iterations stop (before x is read)
    auto finish_x = [&]() {
        hipLaunchKernelGGL(k_x_finish, dim3(fill_grid), dim3(kWG), 0, stream, st, p0, p1, x, n);
        hipLaunchKernelGGL(k_x_finish_clear, dim3(1), dim3(64), 0, stream, st);
    };
    // before the host reads st: take a pending update decision in place
    auto commit = [&]() {
        FinishArgs g = fu;
        g.nparts = La.grid;
        if (M) hipLaunchKernelGGL((k_finish_commit<FIN_PCG_UPDATE>), dim3(1), dim3(kWG), 0, stream, g);
        else hipLaunchKernelGGL((k_finish_commit<FIN_PCG_UPDATE_I>), dim3(1), dim3(kWG), 0, stream, g);
    };
    auto read_state = [&](PcgState &h) -> int {
        commit();
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&h, st, sizeof(PcgState), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        return BJP_OK;
    };

    // r = b - A x and its norms (the panel copy serves it too when built)
    auto resid_product = [&](int phase) {
        sa.resid_phase = phase;
        if (panels) {
            SpmvArgs saf = sa;
            saf.chunk = Lf.chunk;
            hipLaunchKernelGGL(k_spmv_panels<SPMV_RESID>, dim3(panel_grid), dim3(kWG), 0, stream, sa, pa);
            hipLaunchKernelGGL(k_panel_finish<SPMV_RESID>, dim3(Lf.grid), dim3(kWG), 0, stream, saf, pa);
        } else {
            launch_spmv<SPMV_RESID>(gs, Ls.grid, sa, stream);
        }
        return panels ? Lf.grid : Ls.grid;
    };
    if (o.x0_given) {
        finish<FIN_RESID_START>(fa, resid_product(0), stream);
    } else {
        const int zgrid = round8(std::min(ceil_div(n, 8 * kWG), kMaxRedWG));
        hipLaunchKernelGGL(k_start_zero, dim3(zgrid), dim3(kWG), 0, stream, b, r, partials, n);
        finish<FIN_RESID_START>(fa, zgrid, stream);
    }
    start_direction();

    // Polls overlap the iterations: the next batch is launched before the
    // state copied after the previous batch is examined, so the GPU does not
    // wait for the host.  Iterations launched after convergence return at
    // once.  Batch sizes follow the observed convergence rate.
    // Without allocation the slots are ordinary host memory and a poll waits
    // for the whole stream: the launches of the next batch are already
    // queued, so the GPU still runs ahead of the host by one batch.
    PcgState local_slots[2];
    PcgState *hs = no_alloc ? local_slots : pinned_states();
    if (!hs) return fail(BJP_EHIP);
    EventPair ev;
    if (!no_alloc) {
        HIP_TRY(hipEventCreateWithFlags(&ev.e[0], hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&ev.e[1], hipEventDisableTiming));
    }
    auto post = [&](int slot) -> int {
        commit();
        HIP_TRY(hipMemcpyAsync(&hs[slot], st, sizeof(PcgState), hipMemcpyDeviceToHost, stream));
        if (!no_alloc) HIP_TRY(hipEventRecord(ev.e[slot], stream));
        return BJP_OK;
    };
    auto take = [&](int slot, PcgState &out) -> int {
        HIP_TRY(hipGetLastError());
        if (no_alloc) HIP_TRY(hipStreamSynchronize(stream));
        else HIP_TRY(hipEventSynchronize(ev.e[slot]));
        out = hs[slot];
        return BJP_OK;
    };

    PcgState h{};
    int replacements = 0, polls = 0, status = BJP_OK;
    int cur = 0, inflight = o.check_every;
    double prev_rel = -1.0;
    int prev_it = 0;
    for (int c = 0; c < inflight; ++c) iteration();
    if ((s = post(0)) != BJP_OK) return fail(s);
    int next = o.check_every;
    for (;;) {
        for (int c = 0; c < next; ++c) iteration();
        if ((s = post(cur ^ 1)) != BJP_OK) return fail(s);
        const int launched_after = next;
        if ((s = take(cur, h)) != BJP_OK) return fail(s);
        ++polls;
        cur ^= 1;
        if (!h.done) {
            // size the batch after the one in flight from the convergence rate
            next = o.check_every;
            if (prev_rel > 0.0 && h.relres > 0.0 && h.it > prev_it && h.relres < prev_rel) {
                const double rate = std::log(h.relres / prev_rel) / (h.it - prev_it);
                const double remain = std::log(o.tol / h.relres) / rate - launched_after;
                if (remain < next) next = std::max(1, (int)std::ceil(remain) + 1);
            }
            prev_rel = h.relres;
            prev_it = h.it;
            continue;
        }
        if (h.status != BJP_OK || h.zero_rhs) break;
        // converged on the recursive residual: confirm with the true one
        finish_x();
        finish<FIN_RESID_TRUE>(fa, resid_product(1), stream);
        if ((s = read_state(h)) != BJP_OK) return fail(s);
        if (h.relres_true <= o.tol) break;
        // a replacement needs an iteration to follow it
        if (replacements >= o.max_replacements || h.it >= o.max_iter) {
            status = BJP_ENOCONV;
            break;
        }
        ++replacements;  // r now holds b - A x: restart the direction from it
        hipLaunchKernelGGL(k_pcg_restart, dim3(1), dim3(64), 0, stream, st);
        start_direction();
        for (int c = 0; c < o.check_every; ++c) iteration();
        cur = 0;
        if ((s = post(0)) != BJP_OK) return fail(s);
        next = o.check_every;
        prev_rel = -1.0;
    }
    if (status == BJP_OK) status = h.status;
    if (h.zero_rhs) {
        hipLaunchKernelGGL(k_fill, dim3(fill_grid), dim3(kWG), 0, stream, x, n, 0.0);
        h.relres_true = 0.0;
        HIP_TRY(hipStreamSynchronize(stream));
    } else if (status != BJP_OK) {
        finish_x();
        finish<FIN_RESID_TRUE>(fa, resid_product(1), stream);
        if ((s = read_state(h)) != BJP_OK) return fail(s);
    }
    info->status = status;
    info->iterations = h.it;
    info->replacements = replacements;
    info->polls = polls;
    info->rel_res_recursive = h.relres;
    info->rel_res_true = h.relres_true;
    return status;
}

// ---------------------------------------------------------------------------
// Static scratch of the allocation-free solver: one copy per GPU, held from
// the library's first use on that GPU until the process ends.  Host code
// never uses the symbol itself as an address: each device's copy is looked
// up once with hipGetSymbolAddress (with that device current) and the
// pointer kept.
// ---------------------------------------------------------------------------
__device__ __align__(256) unsigned char scratch[BJP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
void *scratch_ptrs[kMaxDevices] = {};

// This device's copy of `scratch` (nullptr if the lookup fails).
void *device_scratch() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptrs[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        scratch_ptrs[dev] = p;
    }
    return scratch_ptrs[dev];
}

}  // namespace

extern "C" {

int bjp_pcg_solve(const bjp_csr_t *A, const bjp_precond_t *M, const double *b, double *x,
                  const bjp_pcg_opts_t *opts, void *ws, size_t ws_bytes, bjp_pcg_info_t *info,
                  hipStream_t stream) {
    return pcg_solve_impl(A, M, b, x, opts, ws, ws_bytes, info, stream, false);
}

int bjp_pcg_solve_noalloc(const bjp_csr_t *A, const bjp_precond_t *M, const double *b, double *x,
                          const bjp_pcg_opts_t *opts, bjp_pcg_info_t *info, hipStream_t stream) {
    if (!info) return BJP_EINVAL;
    std::memset(info, 0, sizeof(*info));
    if (check_csr_host(A) != BJP_OK) return info->status = BJP_EINVAL;
    // sizes first: a system beyond the scratch is refused before any HIP call
    const size_t need = pcg_ws_bytes(A, false);
    if (need > (size_t)BJP_NOALLOC_SCRATCH_BYTES) return info->status = BJP_EWORKSPACE;
    void *ws = device_scratch();
    if (!ws) return info->status = BJP_EHIP;
    return pcg_solve_impl(A, M, b, x, opts, ws, BJP_NOALLOC_SCRATCH_BYTES, info, stream, true);
}

int bjp_kappa_workspace(const bjp_csr_t *A, int steps, size_t *bytes) {
    if (!bytes) return BJP_EINVAL;
    *bytes = 0;
    if (check_csr_host(A) != BJP_OK || steps <= 0) return BJP_EINVAL;
    const int n = std::max(A->n, 1);
    const size_t ld = (size_t)((n + 31) & ~31);
    const RowLaunch Lg = gram_shape(n);
    const int redwg = std::max(kMaxRedWG, Lg.grid);
    *bytes = 2 * al256(sizeof(double) * ld * (steps + 1))    // U, V
             + 3 * al256(sizeof(double) * ld)                 // w, r~, z~
             + al256(sizeof(double) * (steps + 1))            // c
             + al256(sizeof(double) * (size_t)Lg.grid * (steps + 1))  // Gram partials
             + 2 * al256(sizeof(double) * steps)              // alpha, beta
             + al256(sizeof(double) * 2 * redwg)              // grid_sum partials
             + al256(sizeof(LanczosState)) + 2 * al256(64);
    return BJP_OK;
}

int bjp_kappa_estimate(const bjp_csr_t *A, const bjp_precond_t *M, const double *v0, int steps,
                       double *alpha, double *beta, void *ws, size_t ws_bytes, bjp_kappa_info_t *info,
                       hipStream_t stream) {
    if (!info) return BJP_EINVAL;
    std::memset(info, 0, sizeof(*info));
    auto fail = [&](int st) {
        info->status = st;
        return st;
    };
    if (check_csr_host(A) != BJP_OK || steps <= 0) return fail(BJP_EINVAL);
    const int n = A->n;
    if (n == 0 || !v0) return fail(BJP_EINVAL);
    if (M && n > 0 && !precond_ok(M, n)) return fail(BJP_EINVAL);
    size_t need = 0;
    bjp_kappa_workspace(A, steps, &need);
    if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255)) return fail(BJP_EWORKSPACE);

    const size_t ld = (size_t)((n + 31) & ~31);
    const RowLaunch Lg = gram_shape(n);
    const int redwg = std::max(kMaxRedWG, Lg.grid);
    Carver cv{static_cast<char *>(ws)};
    double *U = cv.take<double>(ld * (steps + 1));
    double *V = cv.take<double>(ld * (steps + 1));
    double *w = cv.take<double>(ld), *rt = cv.take<double>(ld), *zt = cv.take<double>(ld);
    double *c = cv.take<double>(steps + 1);
    double *cpart = cv.take<double>((size_t)Lg.grid * (steps + 1));
    double *al = cv.take<double>(steps), *be = cv.take<double>(steps);
    double *partials = cv.take<double>(2 * redwg);
    LanczosState *ls = cv.take<LanczosState>(1);
    int32_t *flags = cv.take<int32_t>(16);
    double *zeros = cv.take<double>(8);
    if (!M) {
        V = U;     // M = I: u_j == v_j
        zt = rt;
    }

    int s = run_validate(A, flags, stream);
    if (s != BJP_OK) return fail(s);

    LanczosState h{};
    // Small systems: the whole estimate in one workgroup (small.hpp), the same
    // steps and decisions.
    if (n <= kSmallMaxRows && (long long)A->nnz <= (long long)kSmallMaxMeanRow * n && steps <= kSmallMaxSteps) {
        LanczosSmallArgs la{};
        la.n = n;
        la.nnz = (int)A->nnz;
        la.rp = A->row_ptr;
        la.ci = A->col_idx;
        la.val = A->val;
        if (M) {
            la.nblocks = M->num_blocks;
            la.num_packets = M->num_packets;
            la.uniform_nb = M->block_size;
            la.off = M->offsets;
            la.tiles = M->tiles;
        }
        la.v0 = v0;
        la.steps = steps;
        la.U = U;
        la.V = V;
        la.ld = ld;
        la.alpha = al;
        la.beta = be;
        la.ls = ls;
        launch_lanczos_small(M, la, stream);
        HIP_TRY(hipGetLastError());
    } else {
        const int gs = auto_spmv(A);
        const RowLaunch Ls = spmv_shape(n, gs);
        const RowLaunch Lr = rows_shape(n);
        hipLaunchKernelGGL(k_lanczos_state_init, dim3(1), dim3(64), 0, stream, ls, steps);
        hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, stream, zeros, 8, 0.0);
        HIP_TRY(hipMemcpyAsync(rt, v0, sizeof(double) * n, hipMemcpyDeviceToDevice, stream));

        ApplyArgs aa{};
        aa.n = n;
        if (M) {
            aa.nblocks = M->num_blocks;
            aa.num_packets = M->num_packets;
            aa.uniform_nb = M->block_size;
            aa.off = M->offsets;
            aa.tiles = M->tiles;
        }
        const RowLaunch La = M ? apply_shape(M) : Lr;
        aa.rin = rt;
        aa.zout = zt;
        aa.ls = ls;
        aa.partials = partials;
        FinishArgs fl{};
        fl.ls = ls;
        fl.partials = partials;
        fl.alpha_out = al;
        fl.beta_out = be;
        if (M) launch_apply<APPLY_PLAIN>(M, La.grid, aa, stream);
        hipLaunchKernelGGL(k_lanczos_start, dim3(Lr.grid), dim3(kWG), 0, stream, ls, rt, zt, n, Lr.chunk,
                           partials);
        finish<FIN_LZ_START>(fl, Lr.grid, stream);

        SpmvArgs sa{};
        sa.n = n;
        sa.chunk = Ls.chunk;
        sa.rp = A->row_ptr;
        sa.ci = A->nnz > 0 ? A->col_idx : reinterpret_cast<const int32_t *>(zeros);
        sa.val = A->nnz > 0 ? A->val : zeros;
        sa.ls = ls;
        sa.zt = zt;
        sa.rt = rt;
        sa.V = V;
        sa.U = U;
        sa.ld = ld;
        sa.w = w;
        sa.has_m = M ? 1 : 0;
        sa.partials = partials;

        GramArgs ga{};
        ga.n = n;
        ga.chunk = Lg.chunk;
        ga.ls = ls;
        ga.w = w;
        ga.U = U;
        ga.V = V;
        ga.ld = ld;
        ga.rt = rt;
        ga.c = c;
        ga.cpart = cpart;
        ga.ldc = steps + 1;
        ga.has_m = M ? 1 : 0;
        ga.partials = partials;

        for (int j = 0; j < steps; ++j) {
            launch_spmv<SPMV_LANCZOS>(gs, Ls.grid, sa, stream);
            finish<FIN_LZ_ALPHA>(fl, Ls.grid, stream);
            hipLaunchKernelGGL((k_gram<GRAM_FIRST>), dim3(Lg.grid), dim3(kWG), 0, stream, ga);
            hipLaunchKernelGGL(k_gram_reduce, dim3(j + 1), dim3(kWG), 0, stream, ls, cpart, steps + 1, Lg.grid, c);
            hipLaunchKernelGGL((k_gram<GRAM_SECOND>), dim3(Lg.grid), dim3(kWG), 0, stream, ga);
            hipLaunchKernelGGL(k_gram_reduce, dim3(j + 1), dim3(kWG), 0, stream, ls, cpart, steps + 1, Lg.grid, c);
            hipLaunchKernelGGL((k_gram<GRAM_FINAL>), dim3(Lg.grid), dim3(kWG), 0, stream, ga);
            if (M) {
                launch_apply<APPLY_LANCZOS>(M, La.grid, aa, stream);
                finish<FIN_LZ_BETA>(fl, La.grid, stream);
            } else {
                finish<FIN_LZ_BETA>(fl, Lg.grid, stream);
            }
            HIP_TRY(hipGetLastError());
            if ((j & 31) == 31 && j + 1 < steps) {
                HIP_TRY(hipMemcpyAsync(&h, ls, sizeof(h), hipMemcpyDeviceToHost, stream));
                HIP_TRY(hipStreamSynchronize(stream));
                if (h.done) break;
            }
        }
    }
    {
        const int lds_steps = steps <= kTriLdsSteps ? steps : 0;
        hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(64 * kTriWaves), sizeof(double) * 2 * (size_t)lds_steps, stream,
                           ls, al, be, lds_steps);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(&h, ls, sizeof(h), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (alpha && h.steps_done > 0)
        HIP_TRY(hipMemcpyAsync(alpha, al, sizeof(double) * h.steps_done, hipMemcpyDeviceToDevice, stream));
    if (beta && h.steps_done > 1)
        HIP_TRY(hipMemcpyAsync(beta, be, sizeof(double) * (h.steps_done - 1), hipMemcpyDeviceToDevice,
                               stream));
    HIP_TRY(hipStreamSynchronize(stream));
    info->status = h.status;
    info->steps_done = h.steps_done;
    info->theta_min = h.theta_min;
    info->theta_max = h.theta_max;
    info->kappa = h.kappa;
    return h.status;
}

int bjp_batch_precondition_workspace(const bjp_csr_t *A, const bjp_batch_t *B, int precision,
                                     size_t *bytes) {
    if (!bytes) return BJP_EINVAL;
    *bytes = 0;
    if (check_csr_host(A) != BJP_OK) return BJP_EINVAL;
    if (precision != BJP_FP64 && precision != BJP_FP32_STORE) return BJP_EINVAL;
    BatchPlan P;
    const int st = make_batch_plan(A, B, P);
    if (st != BJP_OK) return st;
    *bytes = batch_precond_bytes(P, precision);
    return BJP_OK;
}

int bjp_batch_precondition(const bjp_csr_t *A, const bjp_batch_t *B, int precision, void *ws,
                           size_t ws_bytes, bjp_batch_precond_t *M_out, int32_t *failed_block,
                           hipStream_t stream) {
    if (failed_block) *failed_block = -1;
    if (!M_out) return BJP_EINVAL;
    std::memset(M_out, 0, sizeof(*M_out));
    if (check_csr_host(A) != BJP_OK) return BJP_EINVAL;
    if (precision != BJP_FP64 && precision != BJP_FP32_STORE) return BJP_EINVAL;
    BatchPlan P;
    int st = make_batch_plan(A, B, P);
    if (st != BJP_OK) return st;
    if (!ws || ws_bytes < batch_precond_bytes(P, precision) || (reinterpret_cast<uintptr_t>(ws) & 255))
        return BJP_EWORKSPACE;
    const int S = B->num_systems;
    const size_t elem = precision == BJP_FP32_STORE ? 4 : 8;
    Carver cv{static_cast<char *>(ws)};
    SysInfo *sys = cv.take<SysInfo>(S);
    int32_t *rows = cv.take<int32_t>(S + 1);
    int32_t *off = cv.take<int32_t>(P.off.size());
    char *tiles = cv.base + cv.used;
    cv.used += al256(P.tile_scalars * elem);
    int32_t *flags = cv.take<int32_t>(16);
    SetupSys *items = cv.take<SetupSys>(S);
    M_out->num_systems = S;
    M_out->precision = precision;
    M_out->systems = sys;
    M_out->tiles = tiles;

    st = run_validate(A, flags, stream);
    if (st != BJP_OK) return st;
    HIP_TRY(hipMemcpyAsync(sys, P.sys.data(), sizeof(SysInfo) * S, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(rows, B->sys_rows, sizeof(int32_t) * (S + 1), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(off, P.off.data(), sizeof(int32_t) * P.off.size(), hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(k_validate_batch, dim3(std::min(S, 4096)), dim3(kWG), 0, stream, S, rows,
                       A->row_ptr, A->col_idx, flags);
    // one setup launch per lane-group width over all its systems' packets
    std::vector<SetupSys> hi;
    std::vector<int> cls_g, cls_begin, cls_packets;
    for (int G = 1; G <= 64; G *= 2) {
        const int begin = (int)hi.size();
        int packets = 0;
        for (int s = 0; s < S; ++s) {
            const SysInfo &si = P.sys[s];
            if (si.G != G) continue;
            hi.push_back(SetupSys{P.off_base[s], si.tile0, si.nblocks, P.block_base[s], packets, 0});
            packets += si.packets;
        }
        if (packets > 0) {
            cls_g.push_back(G);
            cls_begin.push_back(begin);
            cls_packets.push_back(packets);
        }
    }
    HIP_TRY(hipMemcpyAsync(items, hi.data(), sizeof(SetupSys) * hi.size(), hipMemcpyHostToDevice, stream));
    for (size_t c = 0; c < cls_g.size(); ++c) {
        const int count = (c + 1 < cls_g.size() ? cls_begin[c + 1] : (int)hi.size()) - cls_begin[c];
        const SetupArgs sa{A->row_ptr, A->col_idx, A->val, off, 0, tiles, flags, 0};
        if (precision == BJP_FP32_STORE)
            launch_setup_batch<float>(cls_g[c], cls_packets[c], sa, items + cls_begin[c], count, stream);
        else
            launch_setup_batch<double>(cls_g[c], cls_packets[c], sa, items + cls_begin[c], count, stream);
    }
    HIP_TRY(hipGetLastError());
    int32_t h[4];
    HIP_TRY(hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (h[1]) return BJP_EINVAL;
    if (h[0] != INT_MAX) {
        if (failed_block) *failed_block = h[0];
        return BJP_ENOTSPD;
    }
    return BJP_OK;
}

int bjp_batch_pcg_workspace(const bjp_csr_t *A, const bjp_batch_t *B, size_t *bytes) {
    if (!bytes) return BJP_EINVAL;
    *bytes = 0;
    if (check_csr_host(A) != BJP_OK) return BJP_EINVAL;
    BatchPlan P;
    const int st = make_batch_plan(A, B, P);
    if (st != BJP_OK) return st;
    const size_t S = (size_t)B->num_systems;
    size_t nrt = 0, npt = 0;
    batch_tiles_bound(P, 256, &nrt, &npt);
    const size_t nred = round8((int)std::max(nrt, npt));
    *bytes = 5 * al256(sizeof(double) * (size_t)std::max(A->n, 1))  // r, z, p0, p1, q
             + al256(sizeof(PcgState) * S) + al256(sizeof(Tile) * (nrt + npt)) +
             5 * al256(sizeof(int) * S)                                // tile ranges, iteration caps
             + al256(sizeof(int) * S)                                  // restart list
             + al256(sizeof(double) * 2 * nred) + 2 * al256(64);
    return BJP_OK;
}

int bjp_batch_pcg_solve(const bjp_csr_t *A, const bjp_batch_t *B, const bjp_batch_precond_t *M,
                        const double *b, double *x, const bjp_batch_opts_t *opts, void *ws,
                        size_t ws_bytes, bjp_batch_info_t *info, bjp_system_info_t *per_system,
                        hipStream_t stream) {
    if (!info) return BJP_EINVAL;
    std::memset(info, 0, sizeof(*info));
    auto fail = [&](int st) {
        info->status = st;
        return st;
    };
    if (check_csr_host(A) != BJP_OK || !M || !b || !x || A->n <= 0 || A->nnz <= 0) return fail(BJP_EINVAL);
    BatchPlan P;
    int st = make_batch_plan(A, B, P);
    if (st != BJP_OK) return fail(st);
    const int S = B->num_systems;
    if (M->num_systems != S || !M->systems || !M->tiles) return fail(BJP_EINVAL);
    size_t need = 0;
    bjp_batch_pcg_workspace(A, B, &need);
    if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255)) return fail(BJP_EWORKSPACE);
    bjp_batch_opts_t o{};
    if (opts) o = *opts;
    if (!(o.tol > 0.0)) o.tol = 1e-10;
    if (o.max_replacements == 0) o.max_replacements = 3;
    else if (o.max_replacements < 0) o.max_replacements = 0;
    if (o.check_every <= 0) o.check_every = 16;
    // per-system product schedule and tile rows (the batch-wide values where
    // the per-system arrays are absent or hold 0)
    std::vector<int> sys_gs(S), sys_tr(S);
    for (int s = 0; s < S; ++s) {
        const int ln = o.sys_lanes && o.sys_lanes[s] != 0 ? o.sys_lanes[s] : o.lanes;
        const int gs = spmv_schedule(ln, A);
        sys_gs[s] = gs == kStream7 ? 0 : gs;     // one streaming kernel serves both stage sizes
        const int tr = o.sys_tile_rows && o.sys_tile_rows[s] > 0 ? o.sys_tile_rows[s] : o.tile_rows;
        sys_tr[s] = tr > 0 ? std::max(256, tr) : 2048;
    }

    BatchTables T;
    make_batch_tables(P, sys_tr, sys_gs, T);
    const int nrt = (int)T.rt.size(), npt = (int)T.pt.size();
    const int nred = round8(std::max(nrt, npt));
    std::vector<int> caps(S);
    for (int s = 0; s < S; ++s) caps[s] = o.max_iter > 0 ? o.max_iter : std::max(P.sys[s].n, 1);

    Carver cv{static_cast<char *>(ws)};
    double *r = cv.take<double>(A->n), *z = cv.take<double>(A->n);
    double *p0 = cv.take<double>(A->n), *p1 = cv.take<double>(A->n), *q = cv.take<double>(A->n);
    PcgState *states = cv.take<PcgState>(S);
    Tile *tiles = cv.take<Tile>((size_t)nrt + npt);
    int *rtb = cv.take<int>(S), *rte = cv.take<int>(S), *ptb = cv.take<int>(S), *pte = cv.take<int>(S);
    int *capd = cv.take<int>(S);
    int *restart = cv.take<int>(S);
    double *partials = cv.take<double>(2 * (size_t)nred);
    int32_t *flags = cv.take<int32_t>(16);
    double *zeros = cv.take<double>(8);
    (void)zeros;

    st = run_validate(A, flags, stream);
    if (st != BJP_OK) return fail(st);
    std::vector<Tile> all(T.rt);
    all.insert(all.end(), T.pt.begin(), T.pt.end());
    HIP_TRY(hipMemcpyAsync(tiles, all.data(), sizeof(Tile) * all.size(), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(rtb, T.rt_begin.data(), sizeof(int) * S, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(rte, T.rt_end.data(), sizeof(int) * S, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(ptb, T.pt_begin.data(), sizeof(int) * S, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(pte, T.pt_end.data(), sizeof(int) * S, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(capd, caps.data(), sizeof(int) * S, hipMemcpyHostToDevice, stream));
    const int fill_grid = std::min(ceil_div(A->n, kWG), 4096);
    hipLaunchKernelGGL(k_batch_state_init, dim3(std::min(ceil_div(S, kWG), 1024)), dim3(kWG), 0, stream, states,
                       S, o.tol, capd);
    hipLaunchKernelGGL(k_fill, dim3(fill_grid), dim3(kWG), 0, stream, p0, A->n, 0.0);
    hipLaunchKernelGGL(k_fill, dim3(fill_grid), dim3(kWG), 0, stream, p1, A->n, 0.0);

    const TileSpan rows{tiles, 0, nrt, nrt, static_cast<const SysInfo *>(M->systems)};
    const int rgrid = round8(nrt);
    SpmvArgs sa{};
    sa.n = A->n;
    sa.rp = A->row_ptr;
    sa.ci = A->col_idx;
    sa.val = A->val;
    sa.st = states;
    sa.p0 = p0;
    sa.p1 = p1;
    sa.q = q;
    sa.b = b;
    sa.x = x;
    sa.r = r;
    sa.partials = partials;
    ApplyArgs aa{};
    aa.st = states;
    aa.tiles = M->tiles;
    aa.rin = r;
    aa.zout = z;
    aa.x = x;
    aa.r = r;
    aa.q = q;
    aa.p0 = p0;
    aa.p1 = p1;
    aa.partials = partials;
    FinishArgs fa{};
    fa.st = states;
    fa.partials = partials;

    // `ls` is the stream the iteration kernels go to: the caller's stream, or
    // the capture stream while the graph is recorded
    hipStream_t ls = stream;
    auto apply_all = [&](auto mode_tag) {
        constexpr int MODE = decltype(mode_tag)::value;
        for (size_t c = 0; c < T.cls_g.size(); ++c) {
            const TileSpan span{tiles + nrt, T.cls_begin[c], T.cls_end[c], npt,
                                static_cast<const SysInfo *>(M->systems)};
            const int grid = round8(T.cls_end[c] - T.cls_begin[c]);
            if (M->precision == BJP_FP32_STORE) launch_apply_tiles_t<float, MODE>(T.cls_g[c], grid, aa, span, ls);
            else launch_apply_tiles_t<double, MODE>(T.cls_g[c], grid, aa, span, ls);
        }
    };
    // the product over every row tile: one launch per schedule present
    auto spmv_all = [&](auto mode_tag, hipStream_t sl) {
        constexpr int MODE = decltype(mode_tag)::value;
        for (size_t c = 0; c < T.rs_gs.size(); ++c) {
            const TileSpan span{tiles, T.rs_begin[c], T.rs_end[c], nrt, static_cast<const SysInfo *>(M->systems)};
            launch_spmv_tiles<MODE>(T.rs_gs[c], round8(T.rs_end[c] - T.rs_begin[c]), sa, span, sl);
        }
    };
    auto start_direction = [&]() {
        apply_all(std::integral_constant<int, APPLY_INIT>{});
        hipLaunchKernelGGL(k_finish_sys<FIN_PCG_START>, dim3(S), dim3(kWG), 0, ls, fa, ptb, pte, npt);
    };
    auto iteration = [&]() {
        hipLaunchKernelGGL(k_direction_tiles, dim3(rgrid), dim3(kWG), 0, ls, states, z, p0, p1, rows);
        spmv_all(std::integral_constant<int, SPMV_SIGMA>{}, ls);
        hipLaunchKernelGGL(k_finish_sys<FIN_SIGMA>, dim3(S), dim3(kWG), 0, ls, fa, rtb, rte, nrt);
        apply_all(std::integral_constant<int, APPLY_UPDATE>{});
        hipLaunchKernelGGL(k_finish_sys<FIN_PCG_UPDATE>, dim3(S), dim3(kWG), 0, ls, fa, ptb, pte, npt);
    };
    GraphGuard gg;
    auto iterations = [&]() -> int {
        if (gg.exec) {
            HIP_TRY(hipGraphLaunch(gg.exec, stream));
        } else {
            for (int c = 0; c < o.check_every; ++c) iteration();
        }
        return BJP_OK;
    };
    std::vector<PcgState> h(S);
    auto read_states = [&]() -> int {
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(h.data(), states, sizeof(PcgState) * S, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        return BJP_OK;
    };

    // x = 0: r = b without the residual product
    hipLaunchKernelGGL(k_start_zero_tiles, dim3(rgrid), dim3(kWG), 0, stream, b, x, r, partials, rows);
    hipLaunchKernelGGL(k_finish_sys<FIN_RESID_START>, dim3(S), dim3(kWG), 0, stream, fa, rtb, rte, nrt);
    start_direction();

    // The check_every iterations between polls are recorded once into a graph
    // (on a private stream: the caller's may be the null stream, which cannot
    // capture) and replayed on the caller's stream.  Every kernel reads its
    // scalars from the device state, so one recording serves every replay.
    // The graph holds kernel nodes only.  It is recorded after the start
    // launches, so the GPU runs those meanwhile.
    if (!o.eager) {
        HIP_TRY(hipStreamCreateWithFlags(&gg.cap, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(gg.cap, hipStreamCaptureModeThreadLocal));
        ls = gg.cap;
        for (int c = 0; c < o.check_every; ++c) iteration();
        ls = stream;
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamEndCapture(gg.cap, &g));
        const hipError_t e = hipGraphInstantiate(&gg.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIP_TRY(e);
    }

    std::vector<int> repl(S, 0), host_status(S, BJP_OK);
    for (;;) {
        int active = 0;
        for (;;) {
            if ((st = iterations()) != BJP_OK) return fail(st);
            if ((st = read_states()) != BJP_OK) return fail(st);
            active = 0;
            for (int s = 0; s < S; ++s) active += h[s].done ? 0 : 1;
            if (!active) break;
        }
        // true residual of every system; re-open the ones above tol
        sa.resid_phase = 1;
        spmv_all(std::integral_constant<int, SPMV_RESID>{}, stream);
        hipLaunchKernelGGL(k_finish_sys<FIN_RESID_TRUE>, dim3(S), dim3(kWG), 0, stream, fa, rtb, rte, nrt);
        sa.resid_phase = 0;
        if ((st = read_states()) != BJP_OK) return fail(st);
        std::vector<int> again;
        for (int s = 0; s < S; ++s) {
            if (h[s].status != BJP_OK || h[s].zero_rhs || h[s].relres_true <= o.tol) continue;
            if (repl[s] >= o.max_replacements || h[s].it >= caps[s]) {
                host_status[s] = BJP_ENOCONV;
                continue;
            }
            ++repl[s];
            again.push_back(s);
        }
        if (again.empty()) break;
        HIP_TRY(hipMemcpyAsync(restart, again.data(), sizeof(int) * again.size(), hipMemcpyHostToDevice, stream));
        hipLaunchKernelGGL(k_batch_restart, dim3(1), dim3(kWG), 0, stream, states, restart, (int)again.size());
        start_direction();
    }
    info->status = BJP_OK;
    std::vector<bjp_system_info_t> out(S);
    for (int s = 0; s < S; ++s) {
        const int sst = h[s].status != BJP_OK ? h[s].status : host_status[s];
        out[s].status = sst;
        out[s].iterations = h[s].it;
        out[s].replacements = repl[s];
        out[s].rel_res_recursive = h[s].relres;
        out[s].rel_res_true = h[s].relres_true;
        if (sst == BJP_OK) info->systems_ok++;
        else if (info->status == BJP_OK) info->status = sst;
        info->total_iterations += h[s].it;
        info->max_iterations = std::max(info->max_iterations, h[s].it);
        info->max_rel_res_true = std::max(info->max_rel_res_true, h[s].relres_true);
    }
    if (per_system) std::memcpy(per_system, out.data(), sizeof(bjp_system_info_t) * S);
    return info->status;
}

int bjp_value_grad(const bjp_csr_t *A, const double *lambda, const double *x, double *grad,
                   hipStream_t stream) {
    if (check_csr_host(A) != BJP_OK) return BJP_EINVAL;
    if (A->n == 0 || A->nnz == 0) return BJP_OK;
    if (!lambda || !x || !grad) return BJP_EINVAL;
    const int gs = auto_lanes(A);
    const int rows_per_step = kWG / gs;
    const int grid = round8(std::min(ceil_div(A->n, rows_per_step * 4), 8192));
    const int chunk = ceil_div(A->n, grid);
    switch (gs) {
#define BJP_VG(G)                                                                                   \
    case G:                                                                                         \
        hipLaunchKernelGGL((k_value_grad<G>), dim3(grid), dim3(kWG), 0, stream, A->n, chunk,        \
                           A->row_ptr, A->col_idx, lambda, x, grad);                                 \
        break;
        BJP_VG(1) BJP_VG(2) BJP_VG(4) BJP_VG(8) BJP_VG(16) BJP_VG(32)
        default:
            hipLaunchKernelGGL((k_value_grad<64>), dim3(grid), dim3(kWG), 0, stream, A->n, chunk, A->row_ptr,
                               A->col_idx, lambda, x, grad);
#undef BJP_VG
    }
    HIP_TRY(hipGetLastError());
    return BJP_OK;
}

}  // extern "C"
