// Batched ragged form: many independent sequences of different model
// family, particle count N and length T advance one time step per launch.
//
// A plan holds one SeqDesc per sequence (its model constants and the device
// arrays of its run) and, per time step t, the list of sequences with
// T_s >= t in descending order of per-step cost N^2 L (longest-processing-
// time first).  Each step is two launches: k_batch_prep writes the step's
// StepArgs for every active sequence, then the persistent k_batch_step
// grid pulls those items from an atomic counter, one sequence step per
// workgroup at a time, and runs the FP32 matrix-core step body of the
// item's model family.  A final k_backtrack_ragged recovers every MAP path.
#pragma once

#include "smsq_mfma.hpp"

namespace smsq {

// Model families the batched kernel carries, by dispatch code: the first
// four codes equal the model kinds (GROWTH1D d 1, RANGE2D 2, CV4D 4, ARM7 7,
// the families of the learned proposal), then the pose family (d 3) and the
// linear-Gaussian family at d = 2.
constexpr int kCodeSE2 = 4, kCodeLinGauss2 = 5;
constexpr int kBatchFamilies = 6;

struct SeqDesc {
    DevModel<float> m;
    const float *x0;        // [d] known initial state
    const float *z;         // [T][obs_dim]
    const uint8_t *mask;    // [T][n_obs] or null
    float *parts;           // [T][n][d] particles after each step
    float *phis;            // [T][n] forward-recursion scores
    int32_t *psis;          // [T][n] backpointers
    float *xmap;            // [T + 1][d] MAP path out
    float *logpost;         // [1] J out
    int32_t *idx;           // [T] MAP indices (plan storage)
    int n, T, d, code;
    int n_iter, bw_mode, trans_mode, use_proposal, weights;  // weights 1: log w_j = phi_{t-1}(j)
    float step, bw_scale;
    uint64_t seed;
};

// Writes StepArgs for the count active sequences list[0..count) of step t.
__global__ void k_batch_prep(const SeqDesc *__restrict__ seqs, const int *__restrict__ list, int count, int t,
                             StepArgs<float> *__restrict__ items, uint8_t *__restrict__ codes, uint32_t *status)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const SeqDesc &s = seqs[list[k]];
    StepArgs<float> a;
    a.m = s.m;
    const long nd = (long)s.n * s.d;
    a.x_prev = t == 1 ? s.x0 : s.parts + (long)(t - 2) * nd;
    a.x_prev_stride = 0;
    a.phi_prev = t == 1 ? nullptr : s.phis + (long)(t - 2) * s.n;
    a.log_w = s.weights == 1 ? a.phi_prev : nullptr; a.log_w_stride = 0;
    a.phi_prev_stride = 0;
    a.z = s.z + (long)(t - 1) * s.m.obs_dim; a.z_stride = 0;
    a.mask = s.mask ? s.mask + (long)(t - 1) * s.m.n_obs : nullptr; a.mask_stride = 0;
    a.x = s.parts + (long)(t - 1) * nd; a.x_stride = 0;
    a.phi = s.phis + (long)(t - 1) * s.n; a.phi_stride = 0;
    a.psi = s.psis + (long)(t - 1) * s.n; a.psi_stride = 0;
    a.flags = nullptr; a.flags_stride = 0;
    a.h_out = nullptr; a.h_stride = 0;
    a.status = status;
    a.n_prev = t == 1 ? 1 : s.n;
    a.n = s.n;
    a.t = t;
    a.n_iter = s.n_iter;
    a.bw_mode = s.bw_mode;
    a.trans_mode = s.trans_mode;
    a.init_given = 0;  // the learned proposal, when used, sets it per step
    a.kernel = 0;
    a.do_svgd = 1;
    a.do_viterbi = 1;
    a.step = s.step;
    a.bw_scale = s.bw_scale;
    a.tie_tol = 0.f;
    a.seed = s.seed;
    a.seq_offset = 0;
    items[k] = a;
    codes[k] = (uint8_t)s.code;
}

// Persistent step: workgroups take items in list order until the counter
// passes count (every workgroup reaches the exit).  TS task slots per wave:
// a workgroup of W waves takes sequences of up to 64 W TS particles.
template <int TS>
__device__ __forceinline__ void batch_step_loop(const StepArgs<float> *__restrict__ items,
                                                const uint8_t *__restrict__ codes, int count, uint32_t *counter)
{
    __shared__ int cur;
    for (;;) {
        if (threadIdx.x == 0) cur = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int k = cur;
        __syncthreads();
        if (k >= count) break;
        const StepArgs<float> &a = items[k];
        const bool split = MfmaLds(a.n, a.n_prev, (int)(blockDim.x >> 6)).ns_max > 1;
        switch (codes[k] + (split ? kBatchFamilies : 0)) {
        case GROWTH1D: step_mfma_body<GROWTH1D, 1, TS, false>(a, 0); break;
        case RANGE2D: step_mfma_body<RANGE2D, 2, TS, false>(a, 0); break;
        case CV4D: step_mfma_body<CV4D, 4, TS, false>(a, 0); break;
        case ARM7: step_mfma_body<ARM7, 7, TS, false>(a, 0); break;
        case kCodeSE2: step_mfma_body<SE2, 3, TS, false>(a, 0); break;
        case kCodeLinGauss2: step_mfma_body<LINGAUSS, 2, TS, false>(a, 0); break;
        case kBatchFamilies + GROWTH1D: step_mfma_body<GROWTH1D, 1, TS, true>(a, 0); break;
        case kBatchFamilies + RANGE2D: step_mfma_body<RANGE2D, 2, TS, true>(a, 0); break;
        case kBatchFamilies + CV4D: step_mfma_body<CV4D, 4, TS, true>(a, 0); break;
        case kBatchFamilies + kCodeSE2: step_mfma_body<SE2, 3, TS, true>(a, 0); break;
        case kBatchFamilies + kCodeLinGauss2: step_mfma_body<LINGAUSS, 2, TS, true>(a, 0); break;
        default: step_mfma_body<ARM7, 7, TS, true>(a, 0); break;
        }
        __syncthreads();  // LDS is reused by the next item
    }
}

__global__ __launch_bounds__(1024) void k_batch_step_w16(const StepArgs<float> *__restrict__ items,
                                                         const uint8_t *__restrict__ codes, int count,
                                                         uint32_t *counter)
{
    batch_step_loop<1>(items, codes, count, counter);
}

__global__ __launch_bounds__(512) void k_batch_step_w8(const StepArgs<float> *__restrict__ items,
                                                       const uint8_t *__restrict__ codes, int count,
                                                       uint32_t *counter)
{
    batch_step_loop<2>(items, codes, count, counter);
}

// Backtrack of every sequence (one wave each): i_T = lowest argmax phi_T,
// then the backpointers; J = phi_T(i_T); xmap[0] = x0, xmap[t] = x_t^{i_t}.
__global__ __launch_bounds__(64) void k_backtrack_ragged(const SeqDesc *__restrict__ seqs, int count,
                                                         uint32_t *status)
{
    const int s = blockIdx.x;
    if (s >= count) return;
    const SeqDesc &q = seqs[s];
    const int lane = threadIdx.x, n = q.n, T = q.T, d = q.d;
    const float *ph = q.phis + (long)(T - 1) * n;
    ArgBest<float> ab{-__builtin_huge_valf(), -__builtin_huge_valf(), 0x7fffffff};
    for (int i = lane; i < n; i += kWave) {
        const float v = ph[i];
        if (i == lane) { ab.best = v; ab.arg = i; }
        else argbest_push(ab, v, i);
    }
    ab = wave_argbest(ab);
    if (lane == 0) {
        int cur = ab.arg;
        q.idx[T - 1] = cur;
        for (int t = T; t >= 2; --t) {
            int prev = q.psis[(long)(t - 1) * n + cur];
            if (prev < 0 || prev >= n) { atomicOr(status, STATUS_NONFINITE); prev = 0; }
            q.idx[t - 2] = prev;
            cur = prev;
        }
        q.logpost[0] = ab.best;
        if (!__builtin_isfinite(ab.best)) atomicOr(status, STATUS_NONFINITE);
    }
    __syncthreads();
    for (int c = lane; c < d; c += kWave) q.xmap[c] = q.x0[c];
    for (int e = lane; e < T * d; e += kWave) {
        const int t = e / d, c = e % d;
        q.xmap[(long)(t + 1) * d + c] = q.parts[((long)t * n + q.idx[t]) * d + c];
    }
}

} // namespace smsq
