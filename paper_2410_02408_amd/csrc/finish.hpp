// Finish kernels: one workgroup that sums the per-workgroup partials of the
// preceding launch (fixed order) and takes the solver's scalar decisions.
// Running them as separate launches gives the totals device-wide visibility
// at the kernel boundary, with no fences inside the streaming kernels.
#pragma once

#include "common.hpp"

namespace bjp {

enum FinishOp {
    FIN_SIGMA = 0,         // q0 = p^T A p                -> alpha = rho / sigma
    FIN_RESID_START = 1,   // q0 = b^T b, q1 = r^T r      -> ||b||, start-of-solve checks
    FIN_RESID_TRUE = 2,    // q0 = b^T b, q1 = r^T r      -> true relative residual
    FIN_PCG_START = 3,     // q0 = r^T z                  -> rho, beta = 0
    FIN_PCG_UPDATE = 4,    // q0 = r^T z, q1 = r^T r      -> convergence, beta
    FIN_PCG_UPDATE_I = 5,  // q0 = r^T r (M = I)          -> convergence, beta
    FIN_LZ_START = 6,      // q0 = r^T z                  -> 1 / beta_0
    FIN_LZ_ALPHA = 7,      // q0 = v_j^T A v_j            -> alpha_j
    FIN_LZ_BETA = 8        // q0 = r~^T z~                -> beta_j, next step or stop
};

struct FinishArgs {
    PcgState *st;
    LanczosState *ls;
    const double *partials;
    int nparts;
    double *hist;          // optional PCG residual history
    double *alpha_out;     // Lanczos tridiagonal
    double *beta_out;
};

__device__ __forceinline__ void pcg_after_init(PcgState *st, double rz) {
    if (!(rz > 0.0)) {
        st->status = isfinite(rz) ? BJP_EBREAKDOWN : BJP_ENONFINITE;
        st->done = 1;
    } else {
        st->rho = rz;
        st->beta = 0.0;
    }
}

__device__ __forceinline__ void pcg_after_update(PcgState *st, double rz, double rr, double *hist) {
    const int it = st->it + 1;
    st->it = it;
    const double relres = sqrt(rr) / sqrt(st->bnorm2);
    st->relres = relres;
    if (hist) hist[it] = relres;
    if (!isfinite(rr)) {
        st->status = BJP_ENONFINITE;
        st->done = 1;
    } else if (relres <= st->tol) {
        st->done = 1;
    } else if (!(rz > 0.0)) {
        st->status = isfinite(rz) ? BJP_EBREAKDOWN : BJP_ENONFINITE;
        st->done = 1;
    } else {
        st->beta = rz / st->rho;
        st->rho = rz;
        if (it >= st->max_iter) {
            st->status = BJP_ENOCONV;
            st->done = 1;
        }
    }
}

__device__ __forceinline__ void lanczos_after_beta(LanczosState *ls, double bb, double *beta_out) {
    const int j = ls->j;
    ls->steps_done = j + 1;
    if (!isfinite(bb)) {
        ls->status = BJP_ENONFINITE;
        ls->done = 1;
        return;
    }
    const double b = sqrt(bb > 0.0 ? bb : 0.0);
    if (j + 1 == ls->steps || b <= 1e-12 * ls->scale) {
        ls->done = 1;
        return;
    }
    if (b > ls->scale) ls->scale = b;
    beta_out[j] = b;
    ls->invb = 1.0 / b;
    ls->beta_prev = b;
    ls->j = j + 1;
}

template <int OP>
constexpr int finish_nq() {
    return (OP == FIN_RESID_START || OP == FIN_RESID_TRUE || OP == FIN_PCG_UPDATE) ? 2 : 1;
}

// Whether the decision of OP is taken for a solver in this state.
template <int OP>
__device__ __forceinline__ bool finish_runs(const PcgState *st, const LanczosState *ls) {
    if (OP >= FIN_LZ_START) return !ls->done;
    if (OP == FIN_RESID_TRUE) return true;
    return !st->done;
}

constexpr bool is_update_op(int op) { return op == FIN_PCG_UPDATE || op == FIN_PCG_UPDATE_I; }

// The scalar decision of OP from the totals (thread 0 only).
template <int OP>
__device__ __forceinline__ void finish_decide(const FinishArgs &f, PcgState *st, LanczosState *ls,
                                              const double *out) {
    constexpr int NQ = finish_nq<OP>();
    if (OP == FIN_SIGMA) {
        const double sigma = out[0];
        if (!(sigma > 0.0)) {
            st->status = isfinite(sigma) ? BJP_EBREAKDOWN : BJP_ENONFINITE;
            st->done = 1;
        } else {
            st->alpha = st->rho / sigma;
        }
    } else if (OP == FIN_RESID_START) {
        const double bb = out[0], rr = out[NQ - 1];
        st->bnorm2 = bb;
        if (bb == 0.0) {
            st->zero_rhs = 1;
            st->relres = 0.0;
            st->done = 1;
        } else if (!isfinite(bb) || !isfinite(rr)) {
            st->status = BJP_ENONFINITE;
            st->done = 1;
        } else {
            const double relres = sqrt(rr) / sqrt(bb);
            st->relres = relres;
            if (f.hist && st->it == 0) f.hist[0] = relres;
            if (relres <= st->tol) st->done = 1;
        }
    } else if (OP == FIN_RESID_TRUE) {
        const double bb = out[0], rr = out[NQ - 1];
        st->relres_true = (bb > 0.0) ? sqrt(rr) / sqrt(bb) : 0.0;
    } else if (OP == FIN_PCG_START) {
        pcg_after_init(st, out[0]);
    } else if (OP == FIN_PCG_UPDATE) {
        pcg_after_update(st, out[0], out[NQ - 1], f.hist);
        st->pending = 0;
    } else if (OP == FIN_PCG_UPDATE_I) {
        pcg_after_update(st, out[0], out[0], f.hist);
        st->pending = 0;
    } else if (OP == FIN_LZ_START) {
        const double bb = out[0];
        if (!(bb > 0.0)) {
            ls->status = isfinite(bb) ? BJP_EBREAKDOWN : BJP_ENONFINITE;
            ls->done = 1;
        } else {
            ls->invb = 1.0 / sqrt(bb);
        }
    } else if (OP == FIN_LZ_ALPHA) {
        const double al = out[0];
        f.alpha_out[ls->j] = al;
        ls->alpha_j = al;
        if (!isfinite(al)) {
            ls->status = BJP_ENONFINITE;
            ls->steps_done = ls->j + 1;
            ls->done = 1;
        } else if (fabs(al) > ls->scale) {
            ls->scale = fabs(al);
        }
    } else if (OP == FIN_LZ_BETA) {
        lanczos_after_beta(ls, out[0], f.beta_out);
    }
}

template <int OP>
__global__ __launch_bounds__(kWG) void k_finish(FinishArgs f) {
    constexpr int NQ = finish_nq<OP>();
    if (!finish_runs<OP>(f.st, f.ls)) return;
    double out[NQ];
    sum_partials<NQ>(f.partials, f.nparts, out);
    if (threadIdx.x == 0) finish_decide<OP>(f, f.st, f.ls, out);
}

// Update decisions are deferred: the launch that forms r^T z and r^T r marks
// the state pending, and the decision is taken by whichever comes first, the
// prologue of the next direction update or a commit before the host reads
// the state.
template <int OP>
__global__ __launch_bounds__(kWG) void k_finish_commit(FinishArgs f) {
    static_assert(is_update_op(OP), "update decisions only");
    constexpr int NQ = finish_nq<OP>();
    if (!finish_runs<OP>(f.st, f.ls) || !f.st->pending) return;
    double out[NQ];
    sum_partials<NQ>(f.partials, f.nparts, out);
    if (threadIdx.x == 0) finish_decide<OP>(f, f.st, f.ls, out);
}

// The same decision taken redundantly by every thread of a streaming
// launch, as its prologue: each workgroup sums the partials of the previous
// launch in the fixed order of sum_partials, so every thread reaches the
// identical state, which is returned; workgroup 0 records it at dst.  The
// state is read with uniform (scalar) loads, independent of the vector loads
// the launch may already have in flight.  dst must not be src: other
// workgroups may still be reading src.  With mark_pending (the application)
// the recorded state also marks the update the launch is about to form as
// pending and its x update as owed (unless the solve is done); without it (the
// direction update) the owed x update is recorded as applied.  Must be called
// by every thread, once per launch.
// Field-wise copies of the solver state (whole-struct copies leave a private
// stack object behind, which the compiler then places in LDS per thread).
__device__ __forceinline__ PcgState load_state(const PcgState *__restrict__ s) {
    PcgState L;
    L.rho = s->rho;
    L.alpha = s->alpha;
    L.beta = s->beta;
    L.bnorm2 = s->bnorm2;
    L.tol = s->tol;
    L.relres = s->relres;
    L.relres_true = s->relres_true;
    L.it = s->it;
    L.done = s->done;
    L.status = s->status;
    L.max_iter = s->max_iter;
    L.zero_rhs = s->zero_rhs;
    L.pending = s->pending;
    L.xpend = s->xpend;
    L.pad = 0;
    return L;
}
__device__ __forceinline__ void store_state(PcgState *d, const PcgState &L) {
    d->rho = L.rho;
    d->alpha = L.alpha;
    d->beta = L.beta;
    d->bnorm2 = L.bnorm2;
    d->tol = L.tol;
    d->relres = L.relres;
    d->relres_true = L.relres_true;
    d->it = L.it;
    d->done = L.done;
    d->status = L.status;
    d->max_iter = L.max_iter;
    d->zero_rhs = L.zero_rhs;
    d->pending = L.pending;
    d->xpend = L.xpend;
}

template <int OP>
__device__ __forceinline__ PcgState shared_decide(const PcgState *__restrict__ src, PcgState *dst,
                                                  const double *partials, int nparts, double *hist,
                                                  bool mark_pending = false) {
    constexpr int NQ = finish_nq<OP>();
    __shared__ double red[NQ][kWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    PcgState L = load_state(src);
    double acc[NQ];
    thread_partials<NQ>(partials, nparts, acc);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double v = wave_sum(acc[q]);
        if (lane == 0) red[q][wave] = v;
    }
    __syncthreads();
    if (finish_runs<OP>(&L, nullptr) && (!is_update_op(OP) || L.pending)) {
        double out[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double t = 0.0;
            for (int w = 0; w < kWaves; ++w) t += red[q][w];
            out[q] = t;
        }
        FinishArgs f{};
        f.hist = (blockIdx.x == 0 && tid == 0) ? hist : nullptr;
        finish_decide<OP>(f, &L, nullptr, out);
    }
    PcgState R = L;
    if (mark_pending && !L.done) R.pending = R.xpend = 1;
    if (!mark_pending) R.xpend = 0;
    if (blockIdx.x == 0 && tid == 0) store_state(dst, R);
    return L;
}

// Batched form: workgroup s decides for system s from the partials of its
// tiles [begin[s], end[s]) (partials laid out [q][ntiles]).
template <int OP>
__global__ __launch_bounds__(kWG) void k_finish_sys(FinishArgs f, const int *begin, const int *end, int ntiles) {
    constexpr int NQ = finish_nq<OP>();
    PcgState *st = f.st + blockIdx.x;
    if (!finish_runs<OP>(st, nullptr)) return;
    double out[NQ];
    sum_partials_range<NQ>(f.partials, ntiles, begin[blockIdx.x], end[blockIdx.x], out);
    if (threadIdx.x == 0) finish_decide<OP>(f, st, nullptr, out);
}

}  // namespace bjp
