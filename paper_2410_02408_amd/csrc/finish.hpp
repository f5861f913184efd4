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
    } else if (OP == FIN_PCG_UPDATE_I) {
        pcg_after_update(st, out[0], out[0], f.hist);
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
