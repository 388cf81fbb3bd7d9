// C ABI of the Stein-MAP-Seq hot path (declarations and contracts in
// include/smsq.h).  Host code: argument validation, workspace layout, launch
// configuration and dispatch to the templated kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <algorithm>
#include <map>
#include <string>
#include <vector>
#include <type_traits>

#include "smsq.h"
#include "smsq_kernels.hpp"
#include "smsq_wave.hpp"
#include "smsq_mfma.hpp"
#include "smsq_batch.hpp"
#include "smsq_init.hpp"

using namespace smsq;

struct smsq_model_s {
    smsq_model_desc_t desc;
};

namespace {

constexpr long kLdsLimit = 160 * 1024;  // LDS per compute unit on gfx950
constexpr size_t kHeader = 256;         // workspace header (status word at offset 0)

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

smsq_status_t check_desc(const smsq_model_desc_t *d)
{
    if (!d) return SMSQ_ERR_INVALID;
    if (d->d < 1 || d->d > 16) return SMSQ_ERR_INVALID;
    for (int c = 0; c < d->d; ++c)
        if (!finite_pos(d->q_var[c])) return SMSQ_ERR_INVALID;
    switch (d->kind) {
    case SMSQ_MODEL_GROWTH1D:
        if (d->d != 1 || d->obs_dim != 1 || d->n_obs != 1 || !finite_pos(d->params[6])) return SMSQ_ERR_INVALID;
        return SMSQ_OK;
    case SMSQ_MODEL_RANGE2D: {
        const int nb = (int)d->params[1];
        if (d->d != 2 || nb < 1 || nb > 16 || d->obs_dim != nb || d->n_obs != nb || !finite_pos(d->params[0]))
            return SMSQ_ERR_INVALID;
        return SMSQ_OK;
    }
    case SMSQ_MODEL_CV4D:
        if (d->d != 4 || d->n_obs < 1 || d->n_obs > 16 || d->obs_dim != 2 * d->n_obs) return SMSQ_ERR_INVALID;
        if (!finite_pos(d->params[1]) || !(d->params[2] >= 0.0 && d->params[2] < 1.0) || !finite_pos(d->params[3]))
            return SMSQ_ERR_INVALID;
        return SMSQ_OK;
    case SMSQ_MODEL_ARM7:
        if (d->d != 7 || d->obs_dim != 3 || d->n_obs != 1 || !finite_pos(d->params[0])) return SMSQ_ERR_INVALID;
        return SMSQ_OK;
    case SMSQ_MODEL_ARM14:
        if (d->d != 14 || d->obs_dim != 3 || d->n_obs != 1 || !finite_pos(d->params[0])) return SMSQ_ERR_INVALID;
        for (int c = 22; c < 26; ++c)
            if (!std::isfinite(d->params[c])) return SMSQ_ERR_INVALID;
        return SMSQ_OK;
    case SMSQ_MODEL_SE2: {
        const int nl = (int)d->params[5];
        if (d->d != 3 || d->obs_dim != 2 || d->n_obs != 1 || nl < 1 || nl > 8 || (double)nl != d->params[5])
            return SMSQ_ERR_INVALID;
        if (!finite_pos(d->params[3]) || !finite_pos(d->params[4])) return SMSQ_ERR_INVALID;
        for (int c = 0; c < 6 + 2 * nl; ++c)
            if (!std::isfinite(d->params[c])) return SMSQ_ERR_INVALID;
        return SMSQ_OK;
    }
    case SMSQ_MODEL_LINGAUSS:
        if (d->d < 1 || d->d > 4 || d->obs_dim < 1 || d->obs_dim > 4 || d->n_obs != 1) return SMSQ_ERR_INVALID;
        for (int r = 0; r < d->obs_dim; ++r)
            if (!finite_pos(d->params[32 + r])) return SMSQ_ERR_INVALID;
        return SMSQ_OK;
    default:
        return SMSQ_ERR_INVALID;
    }
}

template <typename T> DevModel<T> make_dev_model(const smsq_model_desc_t &d)
{
    DevModel<T> m;
    std::memset(&m, 0, sizeof(m));
    m.kind = d.kind;
    m.d = d.d;
    m.obs_dim = d.obs_dim;
    m.n_obs = d.n_obs;
    double lz = 0.0;
    for (int c = 0; c < 16; ++c) {
        if (c < d.d) {
            const double q = d.q_var[c];
            m.q[c] = (T)q;
            m.inv_q[c] = (T)(1.0 / q);
            m.sqrt_q[c] = (T)std::sqrt(q);
            m.rs[c] = (T)std::sqrt(kLog2e / (2.0 * q));
            lz += std::log(2.0 * kPi * q);
        }
    }
    m.log_z = (T)(-0.5 * lz);
    for (int c = 0; c < 64; ++c) m.p[c] = (T)d.params[c];
    if (d.kind == SMSQ_MODEL_RANGE2D) m.aux[0] = (T)(1.0 / d.params[0]);
    if (d.kind == SMSQ_MODEL_ARM7 || d.kind == SMSQ_MODEL_ARM14)
        for (int i = 0; i < 7; ++i) {
            m.aux[i] = (T)std::cos(d.params[8 + i]);
            m.aux[7 + i] = (T)std::sin(d.params[8 + i]);
        }
    if (d.kind == SMSQ_MODEL_ARM14) {
        m.grow[0] = d.params[23];
        m.grow[1] = d.params[24];
        m.grow[2] = d.params[25];
    }
    if (d.kind == SMSQ_MODEL_SE2) {
        m.aux[0] = (T)(1.0 / d.params[3]);
        m.aux[1] = (T)(1.0 / d.params[4]);
        m.aux[2] = (T)(-std::log(d.params[5]) - 0.5 * std::log(2.0 * kPi * d.params[3]) -
                       0.5 * std::log(2.0 * kPi * d.params[4]));
    }
    if (d.kind == SMSQ_MODEL_GROWTH1D) {
        m.grow[0] = d.params[2];
        m.grow[1] = d.params[3];
        m.grow[2] = d.params[4];
    }
    return m;
}

size_t elem_size(smsq_dtype_t dt) { return dt == SMSQ_F64 ? sizeof(double) : sizeof(float); }

template <typename T> long step_lds_bytes(int n, int n_prev, int d)
{
    return StepLds<T>(n, n_prev, dpad(d)).total;
}

long lds_bytes(smsq_dtype_t dt, int n, int n_prev, int d)
{
    return dt == SMSQ_F64 ? step_lds_bytes<double>(n, n_prev, d) : step_lds_bytes<float>(n, n_prev, d);
}

int step_threads(int n)
{
    int t = ((n + kWave - 1) / kWave) * kWave;
    if (t < kWave) t = kWave;
    if (t > 1024) t = 1024;
    return t;
}

bool step_shape_ok(smsq_dtype_t dt, int n, int n_prev, int d)
{
    if (n < 1 || n_prev < 1) return false;
    if (lds_bytes(dt, n, n_prev, d) > kLdsLimit) return false;
    const int nt = step_threads(n);
    return (n + nt - 1) / nt <= kMaxRowsPerThread;
}

template <typename KernelFn> hipError_t allow_big_lds(KernelFn fn, long static_bytes = 0)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kLdsLimit - static_bytes));
}

// static LDS of the persistent batch kernels (the queue slot), rounded up
constexpr long kBatchStaticLds = 256;

template <typename T, int KIND, int D>
smsq_status_t launch_step_kd(const StepArgs<T> &a, int batch, hipStream_t s)
{
    auto fn = &k_step<T, KIND, D>;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [&] { attr_err = allow_big_lds(fn); });
    if (attr_err != hipSuccess) return SMSQ_ERR_HIP;
    const long lds = step_lds_bytes<T>(a.n, a.n_prev, D);
    hipLaunchKernelGGL(fn, dim3(batch), dim3(step_threads(a.n)), (size_t)lds, s, a);
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

// The FP32 matrix-core kernel takes sequences of 32 to 1024 particles whose
// state fits LDS and which the one-wave kernel does not take (below 32
// particles the vector-ALU kernels are faster).  The option step_kernel =
// SMSQ_STEP_VALU selects the workgroup vector-ALU kernel for every size,
// SMSQ_STEP_MFMA the matrix-core kernel for every size that fits it
// (batched plans run it at any size).
constexpr int kMfmaMinParticles = 32;

bool use_mfma(int n, int n_prev, int step_kernel)
{
    if (step_kernel == SMSQ_STEP_VALU) return false;
    const MfmaLds L(n, n_prev);
    const bool fits = L.npad <= kMaxParticles && L.total <= kLdsLimit;
    if (step_kernel == SMSQ_STEP_MFMA) return fits;
    return fits && n >= kMfmaMinParticles;
}

template <int KIND, int D, bool SPLIT>
smsq_status_t launch_mfma_split(const StepArgs<float> &a, int batch, hipStream_t s)
{
    auto fn = &k_step_mfma<KIND, D, SPLIT>;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [&] { attr_err = allow_big_lds(fn); });
    if (attr_err != hipSuccess) return SMSQ_ERR_HIP;
    const MfmaLds L(a.n, a.n_prev);
    hipLaunchKernelGGL(fn, dim3(batch), dim3(L.nwaves * kWave), (size_t)L.total, s, a);
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

// Fewer 64-particle tasks than 16 waves: the split instantiation fills the
// workgroup with waves that share each task's sources.
template <int KIND, int D>
smsq_status_t launch_mfma_kd(const StepArgs<float> &a, int batch, hipStream_t s)
{
    return MfmaLds(a.n, a.n_prev).ns_max > 1 ? launch_mfma_split<KIND, D, true>(a, batch, s)
                                              : launch_mfma_split<KIND, D, false>(a, batch, s);
}

template <typename T, int KIND, int D>
smsq_status_t launch_wave_kd(const StepArgs<T> &a, int batch, hipStream_t s)
{
    hipLaunchKernelGGL((k_step_wave<T, KIND, D>), dim3(batch), dim3(kWave), 0, s, a);
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

// The one-wave kernel fits at most 64 particles and 64 previous ones; by
// default it takes steps of up to 32 particles in both precisions, and of
// up to 40 for FP32 states of one or two dimensions (measured: 8..12%
// faster than the workgroup vector-ALU kernel at 10..20 particles, 2.2x for
// the 14-D model in FP64, even at 32, slower at 64; in FP32 at 32 particles
// 0.70..0.89 of the matrix-core kernel's time, and at 40 for the range
// model 0.73, while the matrix cores win from 40 on for d >= 3 and from 48
// on for d = 2).  step_kernel = SMSQ_STEP_WAVE selects it wherever it fits,
// SMSQ_STEP_VALU or SMSQ_STEP_MFMA the other kernels.
constexpr int kWaveDefaultMax = 32;
constexpr int kWaveSmallStateMax = 40;

bool use_wave(int n, int n_prev, int d, bool fp32, int step_kernel)
{
    if (n > kWaveMaxParticles || n_prev > kWaveMaxParticles) return false;
    if (step_kernel == SMSQ_STEP_WAVE) return true;
    if (step_kernel == SMSQ_STEP_VALU || step_kernel == SMSQ_STEP_MFMA) return false;
    return n <= kWaveDefaultMax || (fp32 && d <= 2 && n <= kWaveSmallStateMax);
}

template <typename T>
smsq_status_t launch_wave(const smsq_model_desc_t &d, const StepArgs<T> &a, int batch, hipStream_t s)
{
    switch (d.kind) {
    case SMSQ_MODEL_GROWTH1D: return launch_wave_kd<T, GROWTH1D, 1>(a, batch, s);
    case SMSQ_MODEL_RANGE2D: return launch_wave_kd<T, RANGE2D, 2>(a, batch, s);
    case SMSQ_MODEL_CV4D: return launch_wave_kd<T, CV4D, 4>(a, batch, s);
    case SMSQ_MODEL_ARM7: return launch_wave_kd<T, ARM7, 7>(a, batch, s);
    case SMSQ_MODEL_SE2: return launch_wave_kd<T, SE2, 3>(a, batch, s);
    case SMSQ_MODEL_ARM14: return launch_wave_kd<T, ARM14, 14>(a, batch, s);
    case SMSQ_MODEL_LINGAUSS:
        switch (d.d) {
        case 1: return launch_wave_kd<T, LINGAUSS, 1>(a, batch, s);
        case 2: return launch_wave_kd<T, LINGAUSS, 2>(a, batch, s);
        case 3: return launch_wave_kd<T, LINGAUSS, 3>(a, batch, s);
        case 4: return launch_wave_kd<T, LINGAUSS, 4>(a, batch, s);
        }
    }
    return SMSQ_ERR_INVALID;
}

template <typename T>
smsq_status_t launch_step(const smsq_model_desc_t &d, const StepArgs<T> &a, int batch, int step_kernel,
                          hipStream_t s);

template <>
smsq_status_t launch_step<float>(const smsq_model_desc_t &d, const StepArgs<float> &a, int batch, int step_kernel,
                                 hipStream_t s)
{
    if (use_wave(a.n, a.n_prev, d.d, true, step_kernel)) return launch_wave<float>(d, a, batch, s);
    // the matrix-core kernel runs the RBF kernel on states of up to 7
    // dimensions; IMQ, Matern and the 14-D model take the vector-ALU kernel
    if (a.kernel == 0 && d.d <= 7 && use_mfma(a.n, a.n_prev, step_kernel)) {
        switch (d.kind) {
        case SMSQ_MODEL_GROWTH1D: return launch_mfma_kd<GROWTH1D, 1>(a, batch, s);
        case SMSQ_MODEL_RANGE2D: return launch_mfma_kd<RANGE2D, 2>(a, batch, s);
        case SMSQ_MODEL_CV4D: return launch_mfma_kd<CV4D, 4>(a, batch, s);
        case SMSQ_MODEL_ARM7: return launch_mfma_kd<ARM7, 7>(a, batch, s);
        case SMSQ_MODEL_SE2: return launch_mfma_kd<SE2, 3>(a, batch, s);
        case SMSQ_MODEL_LINGAUSS:
            switch (d.d) {
            case 1: return launch_mfma_kd<LINGAUSS, 1>(a, batch, s);
            case 2: return launch_mfma_kd<LINGAUSS, 2>(a, batch, s);
            case 3: return launch_mfma_kd<LINGAUSS, 3>(a, batch, s);
            case 4: return launch_mfma_kd<LINGAUSS, 4>(a, batch, s);
            }
        }
        return SMSQ_ERR_INVALID;
    }
    switch (d.kind) {
    case SMSQ_MODEL_GROWTH1D: return launch_step_kd<float, GROWTH1D, 1>(a, batch, s);
    case SMSQ_MODEL_RANGE2D: return launch_step_kd<float, RANGE2D, 2>(a, batch, s);
    case SMSQ_MODEL_CV4D: return launch_step_kd<float, CV4D, 4>(a, batch, s);
    case SMSQ_MODEL_ARM7: return launch_step_kd<float, ARM7, 7>(a, batch, s);
    case SMSQ_MODEL_SE2: return launch_step_kd<float, SE2, 3>(a, batch, s);
    case SMSQ_MODEL_ARM14: return launch_step_kd<float, ARM14, 14>(a, batch, s);
    case SMSQ_MODEL_LINGAUSS:
        switch (d.d) {
        case 1: return launch_step_kd<float, LINGAUSS, 1>(a, batch, s);
        case 2: return launch_step_kd<float, LINGAUSS, 2>(a, batch, s);
        case 3: return launch_step_kd<float, LINGAUSS, 3>(a, batch, s);
        case 4: return launch_step_kd<float, LINGAUSS, 4>(a, batch, s);
        }
    }
    return SMSQ_ERR_INVALID;
}

template <>
smsq_status_t launch_step<double>(const smsq_model_desc_t &d, const StepArgs<double> &a, int batch, int step_kernel,
                                  hipStream_t s)
{
    if (use_wave(a.n, a.n_prev, d.d, false, step_kernel)) return launch_wave<double>(d, a, batch, s);
    switch (d.kind) {
    case SMSQ_MODEL_GROWTH1D: return launch_step_kd<double, GROWTH1D, 1>(a, batch, s);
    case SMSQ_MODEL_RANGE2D: return launch_step_kd<double, RANGE2D, 2>(a, batch, s);
    case SMSQ_MODEL_CV4D: return launch_step_kd<double, CV4D, 4>(a, batch, s);
    case SMSQ_MODEL_ARM7: return launch_step_kd<double, ARM7, 7>(a, batch, s);
    case SMSQ_MODEL_SE2: return launch_step_kd<double, SE2, 3>(a, batch, s);
    case SMSQ_MODEL_ARM14: return launch_step_kd<double, ARM14, 14>(a, batch, s);
    case SMSQ_MODEL_LINGAUSS:
        switch (d.d) {
        case 1: return launch_step_kd<double, LINGAUSS, 1>(a, batch, s);
        case 2: return launch_step_kd<double, LINGAUSS, 2>(a, batch, s);
        case 3: return launch_step_kd<double, LINGAUSS, 3>(a, batch, s);
        case 4: return launch_step_kd<double, LINGAUSS, 4>(a, batch, s);
        }
    }
    return SMSQ_ERR_INVALID;
}

// LDS of the chip-wide particle-mode forward recursion: the scaled means
// table [n_prev][dpad(d)] and phi_{t-1} [n_prev]
template <typename T> long wide_lds_bytes(int n_prev, int d)
{
    return align16((long)n_prev * dpad(d) * sizeof(T)) + (long)n_prev * sizeof(T);
}

// 16 waves per workgroup for states of up to 8 dimensions (one means table
// for all of them, eight rows at a time, two waves per row), 4 for larger
// states (register budget)
constexpr int wide_threads(int d) { return d <= 8 ? 1024 : 256; }
constexpr int kWideMaxBlocks = 512;
constexpr long kWideStaticLds = 512;   // the kernel's row-merge slots (FP64: 320 bytes), rounded up

template <typename T, int KIND, int D, bool FLAGS>
smsq_status_t launch_viterbi_wide_flags(const smsq_model_desc_t &d, int t, int n, int n_prev, const void *x_prev,
                                        const void *phi_prev, const void *z, const uint8_t *mask, const void *x,
                                        void *phi, int32_t *psi, uint8_t *flags, double tie_tol, uint32_t *status,
                                        hipStream_t s)
{
    constexpr int NT = wide_threads(D);
    auto fn = &k_viterbi_particle_wide<T, KIND, D, NT, FLAGS>;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [&] { attr_err = allow_big_lds(fn, kWideStaticLds); });
    if (attr_err != hipSuccess) return SMSQ_ERR_HIP;
    const int rows_per_block = NT / kWave / 2;
    const int grid = std::min((n + rows_per_block - 1) / rows_per_block, kWideMaxBlocks);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(NT), (size_t)wide_lds_bytes<T>(n_prev, D), s,
                       make_dev_model<T>(d), t, n, n_prev, (const T *)x_prev, (const T *)phi_prev, (const T *)z,
                       mask, (const T *)x, (T *)phi, psi, flags, (T)tie_tol, status);
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

// the runner-up is tracked only when tie flags are requested
template <typename T, int KIND, int D>
smsq_status_t launch_viterbi_wide_kd(const smsq_model_desc_t &d, int t, int n, int n_prev, const void *x_prev,
                                     const void *phi_prev, const void *z, const uint8_t *mask, const void *x,
                                     void *phi, int32_t *psi, uint8_t *flags, double tie_tol, uint32_t *status,
                                     hipStream_t s)
{
    return flags ? launch_viterbi_wide_flags<T, KIND, D, true>(d, t, n, n_prev, x_prev, phi_prev, z, mask, x, phi,
                                                                psi, flags, tie_tol, status, s)
                 : launch_viterbi_wide_flags<T, KIND, D, false>(d, t, n, n_prev, x_prev, phi_prev, z, mask, x, phi,
                                                                 psi, flags, tie_tol, status, s);
}

template <typename T>
smsq_status_t launch_viterbi_wide(const smsq_model_desc_t &d, int t, int n, int n_prev, const void *x_prev,
                                  const void *phi_prev, const void *z, const uint8_t *mask, const void *x,
                                  void *phi, int32_t *psi, uint8_t *flags, double tie_tol, uint32_t *status,
                                  hipStream_t s)
{
#define SMSQ_WIDE(K, DD) \
    launch_viterbi_wide_kd<T, K, DD>(d, t, n, n_prev, x_prev, phi_prev, z, mask, x, phi, psi, flags, tie_tol, status, s)
    switch (d.kind) {
    case SMSQ_MODEL_GROWTH1D: return SMSQ_WIDE(GROWTH1D, 1);
    case SMSQ_MODEL_RANGE2D: return SMSQ_WIDE(RANGE2D, 2);
    case SMSQ_MODEL_CV4D: return SMSQ_WIDE(CV4D, 4);
    case SMSQ_MODEL_ARM7: return SMSQ_WIDE(ARM7, 7);
    case SMSQ_MODEL_SE2: return SMSQ_WIDE(SE2, 3);
    case SMSQ_MODEL_ARM14: return SMSQ_WIDE(ARM14, 14);
    case SMSQ_MODEL_LINGAUSS:
        switch (d.d) {
        case 1: return SMSQ_WIDE(LINGAUSS, 1);
        case 2: return SMSQ_WIDE(LINGAUSS, 2);
        case 3: return SMSQ_WIDE(LINGAUSS, 3);
        case 4: return SMSQ_WIDE(LINGAUSS, 4);
        }
    }
#undef SMSQ_WIDE
    return SMSQ_ERR_INVALID;
}

// Rows per workgroup pass of the particle-mode forward recursion without tie
// flags: the largest of 16, 8, 4 that still gives each compute unit a
// workgroup (n / RP >= ~240), 4 below that
inline int rows_pass(int n) { return n >= 16 * 240 ? 16 : n >= 8 * 240 ? 8 : 4; }
// its LDS: D + 1 arrays of n_prev entries rounded up to rows_table_align(RP)
inline int rows_npad(int n_prev, int rp)
{
    const int a = rows_table_align(rp);
    return (n_prev + a - 1) / a * a;
}
template <typename T> long rows_lds_bytes(int n, int n_prev, int d)
{
    return (long)(d + 1) * rows_npad(n_prev, rows_pass(n)) * sizeof(T);
}
constexpr long kRowsStaticLds = 6144;   // row-merge slots, runner-ups, observation (FP64: 5472 bytes), rounded up

// states the rows kernel takes: FP32 up to 8 dimensions (no register
// spills); FP64 up to 4, where it still beats the two-waves-per-row kernel
// although from d = 3 it spills (measured, back-to-back launches: clutter
// model N = 512 15.9 against 21.9 us, pose model N = 1000 20.0 against 20.7;
// the 7-D arm at N = 1024 29.8 against 25.5, so d > 4 keeps the other kernel)
template <typename T> constexpr bool rows_fits(int d) { return sizeof(T) == 4 ? d <= 8 : d <= 4; }

template <typename T, int KIND, int D, int RP, bool FLAGS>
smsq_status_t launch_viterbi_rows_rp(const smsq_model_desc_t &d, int t, int n, int n_prev, const void *x_prev,
                                     const void *phi_prev, const void *z, const uint8_t *mask, const void *x,
                                     void *phi, int32_t *psi, uint8_t *flags, double tie_tol, uint32_t *status,
                                     hipStream_t s)
{
    auto fn = &k_viterbi_particle_rows<T, KIND, D, RP, FLAGS>;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [&] { attr_err = allow_big_lds(fn, kRowsStaticLds); });
    if (attr_err != hipSuccess) return SMSQ_ERR_HIP;
    const int npad = rows_npad(n_prev, RP);
    const int grid = std::min((n + RP - 1) / RP, kWideMaxBlocks);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kRowsWaves * kWave), (size_t)rows_lds_bytes<T>(n, n_prev, D), s,
                       make_dev_model<T>(d), t, n, n_prev, npad, (const T *)x_prev, (const T *)phi_prev,
                       (const T *)z, mask, (const T *)x, (T *)phi, psi, flags, (T)tie_tol, status);
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

template <typename T, int KIND, int D, bool FLAGS>
smsq_status_t launch_viterbi_rows_flags(const smsq_model_desc_t &d, int t, int n, int n_prev, const void *x_prev,
                                        const void *phi_prev, const void *z, const uint8_t *mask, const void *x,
                                        void *phi, int32_t *psi, uint8_t *flags, double tie_tol, uint32_t *status,
                                        hipStream_t s)
{
#define SMSQ_ROWS_RP(RP) \
    launch_viterbi_rows_rp<T, KIND, D, RP, FLAGS>(d, t, n, n_prev, x_prev, phi_prev, z, mask, x, phi, psi, flags, \
                                                  tie_tol, status, s)
    switch (rows_pass(n)) {
    case 16: return SMSQ_ROWS_RP(16);
    case 8: return SMSQ_ROWS_RP(8);
    default: return SMSQ_ROWS_RP(4);
    }
#undef SMSQ_ROWS_RP
}

template <typename T, int KIND, int D>
smsq_status_t launch_viterbi_rows_kd(const smsq_model_desc_t &d, int t, int n, int n_prev, const void *x_prev,
                                     const void *phi_prev, const void *z, const uint8_t *mask, const void *x,
                                     void *phi, int32_t *psi, uint8_t *flags, double tie_tol, uint32_t *status,
                                     hipStream_t s)
{
    if constexpr (!rows_fits<T>(D)) {
        return SMSQ_ERR_UNSUPPORTED;
    } else {
        return flags ? launch_viterbi_rows_flags<T, KIND, D, true>(d, t, n, n_prev, x_prev, phi_prev, z, mask, x,
                                                                   phi, psi, flags, tie_tol, status, s)
                     : launch_viterbi_rows_flags<T, KIND, D, false>(d, t, n, n_prev, x_prev, phi_prev, z, mask, x,
                                                                    phi, psi, flags, tie_tol, status, s);
    }
}

template <typename T>
smsq_status_t launch_viterbi_rows(const smsq_model_desc_t &d, int t, int n, int n_prev, const void *x_prev,
                                  const void *phi_prev, const void *z, const uint8_t *mask, const void *x,
                                  void *phi, int32_t *psi, uint8_t *flags, double tie_tol, uint32_t *status,
                                  hipStream_t s)
{
#define SMSQ_ROWS(K, DD) \
    launch_viterbi_rows_kd<T, K, DD>(d, t, n, n_prev, x_prev, phi_prev, z, mask, x, phi, psi, flags, tie_tol, status, s)
    switch (d.kind) {
    case SMSQ_MODEL_GROWTH1D: return SMSQ_ROWS(GROWTH1D, 1);
    case SMSQ_MODEL_RANGE2D: return SMSQ_ROWS(RANGE2D, 2);
    case SMSQ_MODEL_CV4D: return SMSQ_ROWS(CV4D, 4);
    case SMSQ_MODEL_ARM7: return SMSQ_ROWS(ARM7, 7);
    case SMSQ_MODEL_SE2: return SMSQ_ROWS(SE2, 3);
    case SMSQ_MODEL_ARM14: return SMSQ_ROWS(ARM14, 14);
    case SMSQ_MODEL_LINGAUSS:
        switch (d.d) {
        case 1: return SMSQ_ROWS(LINGAUSS, 1);
        case 2: return SMSQ_ROWS(LINGAUSS, 2);
        case 3: return SMSQ_ROWS(LINGAUSS, 3);
        case 4: return SMSQ_ROWS(LINGAUSS, 4);
        }
    }
#undef SMSQ_ROWS
    return SMSQ_ERR_INVALID;
}

bool opts_ok(const smsq_svgd_opts_t *o)
{
    return o && o->n_iter >= 0 && std::isfinite(o->step) && finite_pos(o->bw_scale) &&
           (o->bw_mode == 0 || o->bw_mode == 1) && (o->trans_mode == 0 || o->trans_mode == 1) &&
           o->kernel >= SMSQ_KERNEL_RBF && o->kernel <= SMSQ_KERNEL_MATERN32 && (o->weights == 0 || o->weights == 1) &&
           o->step_kernel >= SMSQ_STEP_AUTO && o->step_kernel <= SMSQ_STEP_COOP;
}

uint32_t *status_ptr(void *ws) { return reinterpret_cast<uint32_t *>(ws); }

// Barrier counters of the exchange areas to zero before a multi-workgroup step.
__global__ void k_coop_reset(char *base, long stride, int batch)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < batch) *(uint32_t *)(base + (long)b * stride) = 0u;
}

template <int KIND, int D>
smsq_status_t launch_coop_kd(const StepArgs<float> &a, int batch, const CoopArgs &c, hipStream_t s)
{
    auto fn = &k_step_mfma_coop<KIND, D>;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [&] { attr_err = allow_big_lds(fn); });
    if (attr_err != hipSuccess) return SMSQ_ERR_HIP;
    const int npad = (a.n + 63) / 64 * 64;
    const MfmaLds L(a.n, a.n_prev, kMaxWaves, npad / 64 / c.G, kCoopWinCap);
    hipLaunchKernelGGL(k_coop_reset, dim3((batch + 63) / 64), dim3(64), 0, s, c.base, c.stride, batch);
    StepArgs<float> aa = a;
    CoopArgs cc = c;
    void *args[] = {(void *)&aa, (void *)&cc};
    // every workgroup of the grid resident at once (the barriers need it)
    if (hipLaunchCooperativeKernel(reinterpret_cast<const void *>(fn), dim3(batch * c.G), dim3(kMaxWaves * kWave),
                                   args, (unsigned)L.total, s) != hipSuccess)
        return SMSQ_ERR_HIP;
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

smsq_status_t launch_coop(const smsq_model_desc_t &d, const StepArgs<float> &a, int batch, const CoopArgs &c,
                          hipStream_t s)
{
    switch (d.kind) {
    case SMSQ_MODEL_GROWTH1D: return launch_coop_kd<GROWTH1D, 1>(a, batch, c, s);
    case SMSQ_MODEL_RANGE2D: return launch_coop_kd<RANGE2D, 2>(a, batch, c, s);
    case SMSQ_MODEL_CV4D: return launch_coop_kd<CV4D, 4>(a, batch, c, s);
    case SMSQ_MODEL_ARM7: return launch_coop_kd<ARM7, 7>(a, batch, c, s);
    }
    return SMSQ_ERR_INVALID;
}

// A stream under graph capture takes no cooperative launch.
bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone;
}

// Generic batched step launch (typed).
template <typename T>
smsq_status_t step_typed(const smsq_model_desc_t &d, int batch, int t, int n_prev, const void *x_prev,
                         long x_prev_stride, const void *log_w, long log_w_stride, const void *phi_prev,
                         long phi_prev_stride, const void *z, long z_stride, const uint8_t *mask,
                         long mask_stride, int n, void *x, long x_stride, int init_given, uint64_t seed,
                         uint32_t seq_offset, const smsq_svgd_opts_t *opts, bool do_svgd, bool do_viterbi,
                         void *phi, long phi_stride, int32_t *psi, long psi_stride, uint8_t *flags,
                         long flags_stride, double tie_tol, void *h_out, long h_stride, void *ws,
                         hipStream_t s, const CoopArgs *coop = nullptr)
{
    StepArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.m = make_dev_model<T>(d);
    a.x_prev = (const T *)x_prev; a.x_prev_stride = x_prev_stride;
    a.log_w = (const T *)log_w; a.log_w_stride = log_w_stride;
    if (!log_w && opts && opts->weights == 1 && phi_prev) {
        // mixture weights from the previous step's forward-recursion scores
        a.log_w = (const T *)phi_prev;
        a.log_w_stride = phi_prev_stride;
    }
    a.phi_prev = (const T *)phi_prev; a.phi_prev_stride = phi_prev_stride;
    a.z = (const T *)z; a.z_stride = z_stride;
    a.mask = mask; a.mask_stride = mask_stride;
    a.x = (T *)x; a.x_stride = x_stride;
    a.phi = (T *)phi; a.phi_stride = phi_stride;
    a.psi = psi; a.psi_stride = psi_stride;
    a.flags = flags; a.flags_stride = flags_stride;
    a.h_out = (T *)h_out; a.h_stride = h_stride;
    a.status = status_ptr(ws);
    a.n_prev = n_prev; a.n = n; a.t = t;
    a.n_iter = opts ? opts->n_iter : 0;
    a.bw_mode = opts ? opts->bw_mode : 0;
    a.trans_mode = opts ? opts->trans_mode : 0;
    a.kernel = opts ? opts->kernel : 0;
    a.init_given = init_given;
    a.do_svgd = do_svgd ? 1 : 0;
    a.do_viterbi = do_viterbi ? 1 : 0;
    a.step = (T)(opts ? opts->step : 0.0);
    a.bw_scale = (T)(opts ? opts->bw_scale : 1.0);
    a.tie_tol = (T)tie_tol;
    a.seed = seed; a.seq_offset = seq_offset;
    if constexpr (std::is_same<T, float>::value)
        if (coop && coop->G > 1) return launch_coop(d, a, batch, *coop, s);
    return launch_step<T>(d, a, batch, opts ? opts->step_kernel : SMSQ_STEP_AUTO, s);
}

smsq_status_t step_dispatch(smsq_dtype_t dt, const smsq_model_desc_t &d, int batch, int t, int n_prev,
                            const void *x_prev, long x_prev_stride, const void *log_w, long log_w_stride,
                            const void *phi_prev, long phi_prev_stride, const void *z, long z_stride,
                            const uint8_t *mask, long mask_stride, int n, void *x, long x_stride,
                            int init_given, uint64_t seed, uint32_t seq_offset, const smsq_svgd_opts_t *opts,
                            bool do_svgd, bool do_viterbi, void *phi, long phi_stride, int32_t *psi,
                            long psi_stride, uint8_t *flags, long flags_stride, double tie_tol, void *h_out,
                            long h_stride, void *ws, hipStream_t s, const CoopArgs *coop = nullptr)
{
    if (dt == SMSQ_F64)
        return step_typed<double>(d, batch, t, n_prev, x_prev, x_prev_stride, log_w, log_w_stride, phi_prev,
                                  phi_prev_stride, z, z_stride, mask, mask_stride, n, x, x_stride, init_given,
                                  seed, seq_offset, opts, do_svgd, do_viterbi, phi, phi_stride, psi, psi_stride,
                                  flags, flags_stride, tie_tol, h_out, h_stride, ws, s);
    return step_typed<float>(d, batch, t, n_prev, x_prev, x_prev_stride, log_w, log_w_stride, phi_prev,
                             phi_prev_stride, z, z_stride, mask, mask_stride, n, x, x_stride, init_given, seed,
                             seq_offset, opts, do_svgd, do_viterbi, phi, phi_stride, psi, psi_stride, flags,
                             flags_stride, tie_tol, h_out, h_stride, ws, s, coop);
}

int device_cus()
{
    static int cus = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
        if (cus <= 0) cus = 1;
    });
    return cus;
}

// ---- multi-workgroup steps (Algorithm 2 drivers) --------------------------
// When a batch leaves most compute units idle (at most a quarter busy with
// one workgroup per sequence) and a sequence has at least 512 particles, the
// FP32 matrix-core step of each sequence runs on G workgroups that own its
// target tasks (k_step_mfma_coop): G is the largest power of two that
// divides the sequence's 64-particle tasks with batch * G within the
// compute units (1: the one-workgroup kernels).  Below 512 particles an
// SVGD iteration of one workgroup (26 us at 256 particles) is too short for
// the two barriers and exchanges per iteration to pay (measured: no gain at
// 256, 1.9x at 512, 3.7x at 1024 for one sequence).  Families of the
// matrix-core drivers with a multi-workgroup kernel: growth, range-only,
// clutter, arm.
constexpr int kCoopMinParticles = 512;
bool coop_family(int kind)
{
    return kind == SMSQ_MODEL_GROWTH1D || kind == SMSQ_MODEL_RANGE2D || kind == SMSQ_MODEL_CV4D ||
           kind == SMSQ_MODEL_ARM7;
}

// force: any shape the multi-workgroup kernel takes (step_kernel =
// SMSQ_STEP_COOP), not only where it pays.
int coop_groups(smsq_dtype_t dt, const smsq_model_desc_t &d, int batch, int n, bool force)
{
    if (dt != SMSQ_F32 || !coop_family(d.kind) || d.d > 7) return 1;
    const int ntasks = (n + 63) / 64;
    const MfmaLds L1(n, n);
    if (L1.npad > kMaxParticles) return 1;
    if (!force && (n < kCoopMinParticles || 4L * batch > device_cus())) return 1;
    int G = 1;
    while (2 * G <= ntasks && ntasks % (2 * G) == 0 && (long)batch * 2 * G <= device_cus()) G *= 2;
    if (G > 1 && (MfmaLds(n, n, kMaxWaves, ntasks / G, kCoopWinCap).total > kLdsLimit ||
                  MfmaLds(n, 1, kMaxWaves, ntasks / G, kCoopWinCap).total > kLdsLimit))
        return 1;
    return G;
}

// The run's scratch in the workspace: header (status word), every step's
// particles, back-pointers, ping-pong scores, MAP indices, and the exchange
// areas of the multi-workgroup steps (coop_groups > 1).
struct RunLayout {
    size_t parts, psi, phi, idx, coop, coop_stride, total;
    int G, G_force;  // workgroups per sequence: automatic choice, largest (forced)
};

RunLayout run_layout(smsq_dtype_t dt, const smsq_model_desc_t &desc, int batch, int T, int n)
{
    RunLayout L;
    size_t o = kHeader;
    const size_t es = elem_size(dt);
    const int d = desc.d;
    L.parts = o; o += align256((size_t)batch * T * n * d * es);
    L.psi = o; o += align256((size_t)batch * T * n * sizeof(int32_t));
    L.phi = o; o += align256((size_t)2 * batch * n * es);
    L.idx = o; o += align256((size_t)batch * T * sizeof(int32_t));
    L.G = coop_groups(dt, desc, batch, n, false);
    L.G_force = coop_groups(dt, desc, batch, n, true);
    L.coop = o;
    L.coop_stride = L.G_force > 1 ? (size_t)CoopLayout((n + 63) / 64 * 64, L.G_force).bytes : 0;
    o += (size_t)batch * L.coop_stride;
    L.total = o;
    return L;
}

bool dtype_ok(smsq_dtype_t dt) { return dt == SMSQ_F32 || dt == SMSQ_F64; }

// ---- batched ragged plans ------------------------------------------------

hipError_t batch_kernel_attrs()
{
    static hipError_t err = hipSuccess;
    static std::once_flag once;
    std::call_once(once, [] {
        err = allow_big_lds(&k_batch_step_w16, kBatchStaticLds);
        if (err == hipSuccess) err = allow_big_lds(&k_batch_step_w8, kBatchStaticLds);
    });
    return err;
}

template <typename P> hipError_t dev_alloc(P **p, size_t count, size_t &total)
{
    *p = nullptr;
    if (count == 0) return hipSuccess;
    const size_t bytes = align256(count * sizeof(P));
    total += bytes;
    return hipMalloc((void **)p, bytes);
}

} // namespace

struct smsq_init_mlp_s {
    int max_batch = 0, adam_t = 0;
    float *P = nullptr, *G = nullptr, *Mo = nullptr, *Ve = nullptr;
    uint16_t *w1b = nullptr, *w2b = nullptr, *w3b = nullptr;
    float *F = nullptr, *anc = nullptr, *scl = nullptr;
    uint16_t *Fb = nullptr;
    float *pre1 = nullptr, *pre2 = nullptr, *out = nullptr, *dout = nullptr, *d2 = nullptr, *d1 = nullptr;
    uint16_t *h1 = nullptr, *h2 = nullptr, *doutb = nullptr, *d2b = nullptr, *d1b = nullptr;
    float *lossv = nullptr;
    size_t bytes = 0;
    void free_all()
    {
        void *ps[] = {P, G, Mo, Ve, w1b, w2b, w3b, F, anc, scl, Fb, pre1, pre2, out, dout, d2, d1,
                      h1, h2, doutb, d2b, d1b, lossv};
        for (void *q : ps)
            if (q) (void)hipFree(q);
    }
};

struct smsq_init_set_s {
    int count = 0, max_n = 0;
    InitExample *ex = nullptr;
};

namespace {

hipError_t zero_alloc_bytes(void **p, size_t bytes, size_t &total)
{
    *p = nullptr;
    bytes = align256(bytes);
    total += bytes;
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) e = hipMemset(*p, 0, bytes);  // at creation, never inside a captured run
    return e;
}

void gemm(int M, int N, int K, const uint16_t *A, long sam, long sak, const uint16_t *B, long sbk, long sbn,
          float *C, long ldc, uint16_t *Cb, long ldcb, const float *bias, const float *pre, long ldpre, int mode,
          hipStream_t s)
{
    const int tiles = ((M + 15) / 16) * ((N + 15) / 16);
    hipLaunchKernelGGL(k_gemm_bf16, dim3((tiles + 3) / 4), dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C,
                       ldc, Cb, ldcb, bias, pre, ldpre, mode);
}

// forward on mlp->Fb (batch rows) into mlp->out
void mlp_forward(smsq_init_mlp_s *m, int B, hipStream_t s)
{
    const int H = kInitHidden;
    gemm(B, H, kInitFeat, m->Fb, kInitFeat, 1, m->w1b, 1, kInitFeat, m->pre1, H, m->h1, H, m->P + kOffB1, nullptr,
         0, 0, s);
    gemm(B, H, H, m->h1, H, 1, m->w2b, 1, H, m->pre2, H, m->h2, H, m->P + kOffB2, nullptr, 0, 0, s);
    gemm(B, kInitOut, H, m->h2, H, 1, m->w3b, 1, H, m->out, kInitOut, nullptr, 0, m->P + kOffB3, nullptr, 0, 1, s);
}

// gradients of sum_e <dout_e, out_e> into mlp->G (dout in mlp->dout)
void mlp_backward(smsq_init_mlp_s *m, int B, hipStream_t s)
{
    const int H = kInitHidden, O = kInitOut;
    hipLaunchKernelGGL(k_to_bf16, dim3((B * O + 255) / 256), dim3(256), 0, s, m->dout, m->doutb, (long)B * O);
    // W3, b3
    gemm(O, H, B, m->doutb, 1, O, m->h2, H, 1, m->G + kOffW3, H, nullptr, 0, nullptr, nullptr, 0, 3, s);
    hipLaunchKernelGGL(k_colsum, dim3((O + 63) / 64), dim3(64), 0, s, B, O, m->dout, (long)O, m->G + kOffB3);
    // through layer 3 and the second ReLU
    gemm(B, H, O, m->doutb, O, 1, m->w3b, H, 1, m->d2, H, m->d2b, H, nullptr, m->pre2, H, 2, s);
    gemm(H, H, B, m->d2b, 1, H, m->h1, H, 1, m->G + kOffW2, H, nullptr, 0, nullptr, nullptr, 0, 3, s);
    hipLaunchKernelGGL(k_colsum, dim3((H + 63) / 64), dim3(64), 0, s, B, H, m->d2, (long)H, m->G + kOffB2);
    // through layer 2 and the first ReLU
    gemm(B, H, H, m->d2b, H, 1, m->w2b, H, 1, m->d1, H, m->d1b, H, nullptr, m->pre1, H, 2, s);
    gemm(H, kInitFeat, B, m->d1b, 1, H, m->Fb, kInitFeat, 1, m->G + kOffW1, kInitFeat, nullptr, 0, nullptr, nullptr,
         0, 3, s);
    hipLaunchKernelGGL(k_colsum, dim3((H + 63) / 64), dim3(64), 0, s, B, H, m->d1, (long)H, m->G + kOffB1);
}

void mlp_features(smsq_init_mlp_s *m, const InitExample *ex, int count, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_features, dim3(count), dim3(kWave), 0, s, ex, count, m->F, m->Fb, m->anc, m->scl);
}

// features, forward and sampler for examples ex[0..count)
smsq_status_t init_propose(smsq_init_mlp_s *m, const InitExample *ex, int count, int max_n, int32_t *used,
                           hipStream_t s)
{
    if (count > m->max_batch) return SMSQ_ERR_INVALID;
    mlp_features(m, ex, count, s);
    mlp_forward(m, count, s);
    hipLaunchKernelGGL(k_mix_sample, dim3((max_n + 255) / 256, count), dim3(256), 0, s, ex, count, m->out, m->anc,
                       m->scl, used);
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

} // namespace

struct smsq_batch_plan_s {
    int count = 0, T_max = 0, max_active = 0, max_n = 0;
    bool proposal_ok = true;              // every sequence of a proposal family
    std::vector<int> list_off, list_cnt;  // per step t - 1
    std::vector<SeqDesc> host;            // per sequence
    SeqDesc *seqs = nullptr;
    int *lists = nullptr;
    StepArgs<float> *items = nullptr;
    uint8_t *codes = nullptr;
    uint32_t *counters = nullptr, *status = nullptr;
    float *parts = nullptr, *phis = nullptr;
    int32_t *psis = nullptr, *idx = nullptr;
    size_t lds = 0, device_bytes = 0;
    int waves = 16;
    double tuned[2] = {0.0, 0.0};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_waves = 0;
    smsq_init_mlp_s *mlp = nullptr;       // learned initial particles (null: predictive)
    InitExample *init_ex = nullptr;       // [max_active]
    int32_t *init_used = nullptr;         // [max_active]
    const smsq_init_mlp_s *graph_mlp = nullptr;

    int grid() const
    {
        int nb = 0;
        const hipError_t e = waves == 16
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_step_w16, 16 * kWave, lds)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_step_w8, 8 * kWave, lds);
        if (e != hipSuccess || nb < 1) nb = 1;
        return std::max(1, std::min(device_cus() * nb, max_active));
    }
    void free_all()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        void *ps[] = {seqs, lists, items, codes, counters, status, parts, phis, psis, idx, init_ex, init_used};
        for (void *q : ps)
            if (q) (void)hipFree(q);
    }
    // One step launch pair (prep + persistent step) for step t.
    smsq_status_t step(int t, hipStream_t s) const
    {
        const int cnt = list_cnt[t - 1];
        if (cnt == 0) return SMSQ_OK;
        hipLaunchKernelGGL(k_batch_prep, dim3((cnt + 63) / 64), dim3(64), 0, s, seqs, lists + list_off[t - 1], cnt,
                           t, items, codes, status);
        if (mlp && t >= 2) {
            hipLaunchKernelGGL(k_init_prep, dim3((cnt + 63) / 64), dim3(64), 0, s, seqs, lists + list_off[t - 1],
                               cnt, t, init_ex);
            const smsq_status_t st = init_propose(mlp, init_ex, cnt, max_n, init_used, s);
            if (st != SMSQ_OK) return st;
            hipLaunchKernelGGL(k_init_apply, dim3((cnt + 63) / 64), dim3(64), 0, s, items, init_ex, init_used, cnt);
        }
        const int g = std::min(grid(), cnt);
        if (waves == 16)
            hipLaunchKernelGGL(k_batch_step_w16, dim3(g), dim3(16 * kWave), lds, s, items, codes, cnt,
                               counters + (t - 1));
        else
            hipLaunchKernelGGL(k_batch_step_w8, dim3(g), dim3(8 * kWave), lds, s, items, codes, cnt,
                               counters + (t - 1));
        return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
    }
    smsq_status_t reset(hipStream_t s) const
    {
        hipLaunchKernelGGL(k_fill_u32, dim3((T_max + 255) / 256), dim3(256), 0, s, counters, 0u, T_max);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, status, 0u, 1);
        return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
    }
    smsq_status_t enqueue(hipStream_t s) const
    {
        smsq_status_t st = reset(s);
        for (int t = 1; st == SMSQ_OK && t <= T_max; ++t) st = step(t, s);
        if (st != SMSQ_OK) return st;
        hipLaunchKernelGGL(k_backtrack_ragged, dim3(count), dim3(kWave), 0, s, seqs, count, status);
        return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
    }
};

namespace {

// the families of the learned proposal (and their plan dispatch codes)
bool batch_family(int kind) { return kind >= SMSQ_MODEL_GROWTH1D && kind <= SMSQ_MODEL_ARM7; }

// a plan's dispatch code of a model, or -1 when plans do not carry it
int batch_code(const smsq_model_desc_t &d)
{
    if (batch_family(d.kind)) return d.kind;
    if (d.kind == SMSQ_MODEL_SE2) return kCodeSE2;
    if (d.kind == SMSQ_MODEL_LINGAUSS && d.d == 2) return kCodeLinGauss2;
    return -1;
}

// Algorithm 2 for `batch` sequences in the scratch memory `ws` (ws_bytes
// bytes, laid out by run_layout): the body of smsq_run_batch, shared with the
// entry point that runs in the library's own device array.
smsq_status_t run_batch_ws(smsq_model_t model, smsq_dtype_t dtype, int batch, int T, int n, const void *x0,
                           const void *z, const uint8_t *z_mask, uint64_t seed, const smsq_svgd_opts_t *opts,
                           void *xmap_out, void *logpost_out, void *particles_out, void *ws, size_t ws_bytes,
                           hipStream_t stream)
{
    if (!model || !dtype_ok(dtype) || batch < 1 || T < 1 || n < 1 || !x0 || !z || !opts_ok(opts) || !xmap_out ||
        !logpost_out)
        return SMSQ_ERR_INVALID;
    const smsq_model_desc_t &d = model->desc;
    const RunLayout L = run_layout(dtype, d, batch, T, n);
    if (!ws || ws_bytes < L.total) return SMSQ_ERR_WORKSPACE;
    if (!step_shape_ok(dtype, n, n, d.d) || !step_shape_ok(dtype, n, 1, d.d)) return SMSQ_ERR_UNSUPPORTED;
    char *w = (char *)ws;
    const size_t es = elem_size(dtype);
    char *parts = particles_out ? (char *)particles_out : w + L.parts;
    int32_t *psi = (int32_t *)(w + L.psi);
    char *phi_buf[2] = {w + L.phi, w + L.phi + (size_t)batch * n * es};
    int32_t *idx = (int32_t *)(w + L.idx);
    const long seq_stride = (long)T * n * d.d;
    const long step_stride = (long)n * d.d;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, status_ptr(ws), 0u, 1);
    if (hipGetLastError() != hipSuccess) return SMSQ_ERR_HIP;
    // several workgroups per sequence while the batch leaves compute units idle
    const int G = opts->step_kernel == SMSQ_STEP_COOP ? L.G_force
                  : opts->step_kernel == SMSQ_STEP_AUTO ? L.G : 1;
    const bool coop = G > 1 && opts->kernel == SMSQ_KERNEL_RBF && !capturing(stream);
    const CoopArgs ca{w + L.coop, (long)L.coop_stride, G, 0};
    for (int t = 1; t <= T; ++t) {
        const void *xp = t == 1 ? x0 : (const void *)(parts + (size_t)(t - 2) * step_stride * es);
        const long xp_stride = t == 1 ? (long)d.d : seq_stride;
        const void *phip = t == 1 ? nullptr : (const void *)phi_buf[(t - 1) & 1];
        const int np = t == 1 ? 1 : n;
        const void *zt = (const char *)z + (size_t)(t - 1) * d.obs_dim * es;
        const uint8_t *mt = z_mask ? z_mask + (size_t)(t - 1) * d.n_obs : nullptr;
        void *xt = parts + (size_t)(t - 1) * step_stride * es;
        const smsq_status_t st = step_dispatch(
            dtype, d, batch, t, np, xp, xp_stride, nullptr, 0, phip, np, zt, (long)T * d.obs_dim, mt,
            (long)T * d.n_obs, n, xt, seq_stride, 0, seed, 0, opts, true, true, phi_buf[t & 1], n,
            psi + (size_t)(t - 1) * n, (long)T * n, nullptr, 0, 0.0, nullptr, 0, ws, stream, coop ? &ca : nullptr);
        if (st != SMSQ_OK) return st;
    }
    return smsq_backtrack(dtype, batch, T, n, d.d, psi, phi_buf[T & 1], idx, logpost_out, parts, x0, xmap_out, ws,
                          ws_bytes, stream);
}



} // namespace

// ---- allocation-free Algorithm 2 ------------------------------------------
// Device memory of smsq_run_sequence_noalloc: one array on every GPU the
// library runs on, held until the process ends.  On the host the array's
// name denotes a host-side stand-in, not a device address; host code uses
// only the address hipGetSymbolAddress returns for the current device.
constexpr size_t kNoallocBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
smsq_status_t scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SMSQ_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_addr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SMSQ_ERR_HIP;
        g_scratch_addr[dev] = ptr;
    }
    *out = g_scratch_addr[dev];
    return SMSQ_OK;
}

// The run's device status word as a status code for the caller.
__global__ void k_status_out(const uint32_t *__restrict__ word, int32_t *__restrict__ out)
{
    if (threadIdx.x == 0)
        out[0] = (word[0] & STATUS_STALLED) ? SMSQ_ERR_HIP : (word[0] & STATUS_NONFINITE) ? SMSQ_ERR_NONFINITE : SMSQ_OK;
}

} // namespace

namespace {

// The tuner's choices for this process, keyed by the device architecture
// (name and compute units) and the plan's shape: every sequence's family,
// size, length, iteration count and proposal switch in plan order, the
// learned-initialisation setting and the number of tuned steps.
struct TuneRecord {
    int waves;
    double ms[2];
};
std::mutex g_tune_mu;
std::map<std::string, TuneRecord> g_tune;

std::string tune_key(const smsq_batch_plan_s *p, int steps)
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return std::string();
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the shape
    auto mix = [&](uint64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (v >> (8 * b)) & 0xffu;
            h *= 1099511628211ull;
        }
    };
    for (const SeqDesc &q : p->host) {
        mix((uint64_t)q.code);
        mix((uint64_t)q.d);
        mix((uint64_t)q.n);
        mix((uint64_t)q.T);
        mix((uint64_t)q.n_iter);
        mix((uint64_t)q.use_proposal);
    }
    mix((uint64_t)(p->mlp != nullptr));
    mix((uint64_t)steps);
    char buf[160];
    snprintf(buf, sizeof buf, "%s/%d/%d/%016llx", prop.gcnArchName, prop.multiProcessorCount, p->count,
             (unsigned long long)h);
    return std::string(buf);
}

} // namespace

extern "C" {

smsq_status_t smsq_model_create(const smsq_model_desc_t *desc, smsq_model_t *out)
{
    if (!out) return SMSQ_ERR_INVALID;
    *out = nullptr;
    const smsq_status_t st = check_desc(desc);
    if (st != SMSQ_OK) return st;
    smsq_model_s *m = new (std::nothrow) smsq_model_s;
    if (!m) return SMSQ_ERR_INVALID;
    m->desc = *desc;
    *out = m;
    return SMSQ_OK;
}

smsq_status_t smsq_model_destroy(smsq_model_t model)
{
    delete model;
    return SMSQ_OK;
}

smsq_status_t smsq_workspace_size(smsq_model_t model, smsq_dtype_t dtype, int batch, int T, int n, size_t *bytes)
{
    if (!model || !bytes || !dtype_ok(dtype) || batch < 1 || T < 1 || n < 1) return SMSQ_ERR_INVALID;
    *bytes = run_layout(dtype, model->desc, batch, T, n).total;
    return SMSQ_OK;
}

int smsq_max_particles(smsq_model_t model, smsq_dtype_t dtype)
{
    if (!model || !dtype_ok(dtype)) return 0;
    int lo = 1, hi = 1 << 16;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (step_shape_ok(dtype, mid, mid, model->desc.d)) lo = mid; else hi = mid - 1;
    }
    return lo;
}

smsq_status_t smsq_svgd_step(smsq_model_t model, smsq_dtype_t dtype, int t, int n_prev, const void *x_prev,
                             const void *log_w_prev, const void *z_t, const uint8_t *z_mask, int n, void *x,
                             const smsq_svgd_opts_t *opts, void *h_out, void *ws, size_t ws_bytes,
                             hipStream_t stream)
{
    if (!model || !dtype_ok(dtype) || t < 1 || n < 1 || n_prev < 1 || !x_prev || !z_t || !x || !opts_ok(opts))
        return SMSQ_ERR_INVALID;
    if (!ws || ws_bytes < kHeader) return SMSQ_ERR_WORKSPACE;
    if (!step_shape_ok(dtype, n, n_prev, model->desc.d)) return SMSQ_ERR_UNSUPPORTED;
    return step_dispatch(dtype, model->desc, 1, t, n_prev, x_prev, 0, log_w_prev, 0, nullptr, 0, z_t, 0, z_mask,
                         0, n, x, 0, 1, 0, 0, opts, true, false, nullptr, 0, nullptr, 0, nullptr, 0, 0.0,
                         h_out, 0, ws, stream);
}

smsq_status_t smsq_viterbi_step(smsq_model_t model, smsq_dtype_t dtype, int t, int n_prev, const void *x_prev,
                                const void *phi_prev, const void *z_t, const uint8_t *z_mask, int n,
                                const void *x, const void *lattice, const void *loglik, void *phi, int32_t *psi,
                                uint8_t *tie_flags, double tie_tol, void *ws, size_t ws_bytes,
                                hipStream_t stream)
{
    if (!dtype_ok(dtype) || n < 1 || n_prev < 1 || !phi_prev || !phi || !psi || !(tie_tol >= 0.0))
        return SMSQ_ERR_INVALID;
    if (!ws || ws_bytes < kHeader) return SMSQ_ERR_WORKSPACE;
    if (lattice) {
        if (!loglik) return SMSQ_ERR_INVALID;
        const int rows_per_block = 2;  // four waves, two per row
        const dim3 grid((n + rows_per_block - 1) / rows_per_block), block(4 * kWave);
        if (dtype == SMSQ_F64)
            hipLaunchKernelGGL(k_viterbi_lattice<double>, grid, block, 0, stream, n, n_prev,
                               (const double *)lattice, (const double *)loglik, (const double *)phi_prev,
                               (double *)phi, psi, tie_flags, tie_tol, status_ptr(ws));
        else
            hipLaunchKernelGGL(k_viterbi_lattice<float>, grid, block, 0, stream, n, n_prev,
                               (const float *)lattice, (const float *)loglik, (const float *)phi_prev,
                               (float *)phi, psi, tie_flags, (float)tie_tol, status_ptr(ws));
        return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
    }
    if (!model || t < 1 || !x_prev || !z_t || !x) return SMSQ_ERR_INVALID;
    // particle mode: chip-wide kernels whose LDS holds the means table; 4..16
    // rows per workgroup pass for the states that fit it, two waves per row
    // for the others
    const smsq_model_desc_t &d = model->desc;
    if (dtype == SMSQ_F64 && rows_fits<double>(d.d) &&
        rows_lds_bytes<double>(n, n_prev, d.d) <= kLdsLimit - kRowsStaticLds)
        return launch_viterbi_rows<double>(d, t, n, n_prev, x_prev, phi_prev, z_t, z_mask, x, phi, psi, tie_flags,
                                           tie_tol, status_ptr(ws), stream);
    if (dtype == SMSQ_F32 && rows_fits<float>(d.d) &&
        rows_lds_bytes<float>(n, n_prev, d.d) <= kLdsLimit - kRowsStaticLds)
        return launch_viterbi_rows<float>(d, t, n, n_prev, x_prev, phi_prev, z_t, z_mask, x, phi, psi, tie_flags,
                                          tie_tol, status_ptr(ws), stream);
    if (dtype == SMSQ_F64) {
        if (wide_lds_bytes<double>(n_prev, d.d) > kLdsLimit - kWideStaticLds) return SMSQ_ERR_UNSUPPORTED;
        return launch_viterbi_wide<double>(d, t, n, n_prev, x_prev, phi_prev, z_t, z_mask, x, phi, psi, tie_flags,
                                           tie_tol, status_ptr(ws), stream);
    }
    if (wide_lds_bytes<float>(n_prev, d.d) > kLdsLimit - kWideStaticLds) return SMSQ_ERR_UNSUPPORTED;
    return launch_viterbi_wide<float>(d, t, n, n_prev, x_prev, phi_prev, z_t, z_mask, x, phi, psi, tie_flags,
                                      tie_tol, status_ptr(ws), stream);
}

smsq_status_t smsq_viterbi_lattice_batch(smsq_dtype_t dtype, int batch, int n, int n_prev, const void *lattice,
                                         const void *loglik, const void *phi_prev, void *phi, int32_t *psi,
                                         uint8_t *tie_flags, double tie_tol, void *ws, size_t ws_bytes,
                                         hipStream_t stream)
{
    if (!dtype_ok(dtype) || batch < 1 || batch > 65535 || n < 1 || n_prev < 1 || !lattice || !loglik ||
        !phi_prev || !phi || !psi || !(tie_tol >= 0.0))
        return SMSQ_ERR_INVALID;
    if (!ws || ws_bytes < kHeader) return SMSQ_ERR_WORKSPACE;
    const int rows_per_block = 2;  // four waves, two per row
    const dim3 grid((n + rows_per_block - 1) / rows_per_block, batch), block(4 * kWave);
    if (dtype == SMSQ_F64)
        hipLaunchKernelGGL(k_viterbi_lattice<double>, grid, block, 0, stream, n, n_prev, (const double *)lattice,
                           (const double *)loglik, (const double *)phi_prev, (double *)phi, psi, tie_flags, tie_tol,
                           status_ptr(ws));
    else
        hipLaunchKernelGGL(k_viterbi_lattice<float>, grid, block, 0, stream, n, n_prev, (const float *)lattice,
                           (const float *)loglik, (const float *)phi_prev, (float *)phi, psi, tie_flags,
                           (float)tie_tol, status_ptr(ws));
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

smsq_status_t smsq_backtrack(smsq_dtype_t dtype, int batch, int T, int n, int d, const int32_t *psi,
                             const void *phi_T, int32_t *idx_out, void *logpost_out, const void *particles,
                             const void *x0, void *xmap_out, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!dtype_ok(dtype) || batch < 1 || T < 1 || n < 1 || !psi || !phi_T || !idx_out || !logpost_out)
        return SMSQ_ERR_INVALID;
    const bool gather = particles && x0 && xmap_out;
    if (gather && (d < 1 || d > 16)) return SMSQ_ERR_INVALID;
    if (!ws || ws_bytes < kHeader) return SMSQ_ERR_WORKSPACE;
    const long psi_b = (long)T * n, parts_b = (long)T * n * d;
    if (dtype == SMSQ_F64)
        hipLaunchKernelGGL(k_backtrack<double>, dim3(batch), dim3(kWave), 0, stream, T, n, d, psi, psi_b,
                           (const double *)phi_T, (long)n, idx_out, (double *)logpost_out,
                           (const double *)particles, parts_b, (const double *)x0,
                           gather ? (double *)xmap_out : nullptr, status_ptr(ws));
    else
        hipLaunchKernelGGL(k_backtrack<float>, dim3(batch), dim3(kWave), 0, stream, T, n, d, psi, psi_b,
                           (const float *)phi_T, (long)n, idx_out, (float *)logpost_out,
                           (const float *)particles, parts_b, (const float *)x0,
                           gather ? (float *)xmap_out : nullptr, status_ptr(ws));
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

smsq_status_t smsq_backtrack_steps(smsq_dtype_t dtype, int T, const int *n_t, int n_max, const int32_t *psi,
                                   const void *phi_T, int32_t *idx_out, void *logpost_out, void *ws,
                                   size_t ws_bytes, hipStream_t stream)
{
    if (!dtype_ok(dtype) || T < 1 || n_max < 1 || !n_t || !psi || !phi_T || !idx_out || !logpost_out)
        return SMSQ_ERR_INVALID;
    if (n_t[0] != 1) return SMSQ_ERR_INVALID;
    for (int t = 1; t <= T; ++t)
        if (n_t[t] < 1 || n_t[t] > n_max) return SMSQ_ERR_INVALID;
    const size_t need = kHeader + sizeof(int) * ((size_t)T + 1);
    if (!ws || ws_bytes < need) return SMSQ_ERR_WORKSPACE;
    int *cnt = reinterpret_cast<int *>(static_cast<unsigned char *>(ws) + kHeader);
    if (hipMemcpyAsync(cnt, n_t, sizeof(int) * ((size_t)T + 1), hipMemcpyHostToDevice, stream) != hipSuccess)
        return SMSQ_ERR_HIP;
    if (dtype == SMSQ_F64)
        hipLaunchKernelGGL(k_backtrack_steps<double>, dim3(1), dim3(kWave), 0, stream, T, cnt, n_max, psi,
                           (const double *)phi_T, idx_out, (double *)logpost_out, status_ptr(ws));
    else
        hipLaunchKernelGGL(k_backtrack_steps<float>, dim3(1), dim3(kWave), 0, stream, T, cnt, n_max, psi,
                           (const float *)phi_T, idx_out, (float *)logpost_out, status_ptr(ws));
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

smsq_status_t smsq_batch_step(smsq_model_t model, smsq_dtype_t dtype, int batch, int t, int n_prev,
                              const void *x_prev, long x_prev_stride, const void *phi_prev, const void *z,
                              long z_stride, const uint8_t *z_mask, long mask_stride, int n, void *x,
                              long x_stride, int init_given, uint64_t seed, uint32_t seq_offset,
                              const smsq_svgd_opts_t *opts, void *phi, int32_t *psi, uint8_t *tie_flags,
                              long out_stride, double tie_tol, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!model || !dtype_ok(dtype) || batch < 1 || t < 1 || n < 1 || n_prev < 1 || !x_prev || !z || !x ||
        !phi || !psi || !opts_ok(opts) || !(tie_tol >= 0.0) || out_stride < n || out_stride < n_prev)
        return SMSQ_ERR_INVALID;
    const smsq_model_desc_t &d = model->desc;
    if (x_stride < (long)n * d.d || (batch > 1 && x_prev_stride < (long)n_prev * d.d) ||
        (batch > 1 && z_stride < d.obs_dim) || (z_mask && batch > 1 && mask_stride < d.n_obs))
        return SMSQ_ERR_INVALID;
    if (t == 1 && n_prev != 1) return SMSQ_ERR_INVALID;
    if (!ws || ws_bytes < kHeader) return SMSQ_ERR_WORKSPACE;
    if (!step_shape_ok(dtype, n, n_prev, model->desc.d)) return SMSQ_ERR_UNSUPPORTED;
    return step_dispatch(dtype, model->desc, batch, t, n_prev, x_prev, x_prev_stride, nullptr, 0, phi_prev,
                         out_stride, z, z_stride, z_mask, mask_stride, n, x, x_stride, init_given, seed, seq_offset,
                         opts, true, true, phi, out_stride, psi, out_stride, tie_flags, out_stride, tie_tol,
                         nullptr, 0, ws, stream);
}

smsq_status_t smsq_run_batch(smsq_model_t model, smsq_dtype_t dtype, int batch, int T, int n, const void *x0,
                             const void *z, const uint8_t *z_mask, uint64_t seed, const smsq_svgd_opts_t *opts,
                             void *xmap_out, void *logpost_out, void *particles_out, void *ws, size_t ws_bytes,
                             hipStream_t stream)
{
    return run_batch_ws(model, dtype, batch, T, n, x0, z, z_mask, seed, opts, xmap_out, logpost_out, particles_out,
                        ws, ws_bytes, stream);
}

smsq_status_t smsq_run_sequence(smsq_model_t model, smsq_dtype_t dtype, int T, int n, const void *x0,
                                const void *z, const uint8_t *z_mask, uint64_t seed, const smsq_svgd_opts_t *opts,
                                void *xmap_out, void *logpost_out, void *particles_out, void *ws, size_t ws_bytes,
                                hipStream_t stream)
{
    return smsq_run_batch(model, dtype, 1, T, n, x0, z, z_mask, seed, opts, xmap_out, logpost_out, particles_out,
                          ws, ws_bytes, stream);
}

smsq_status_t smsq_run_sequence_noalloc(smsq_model_t model, smsq_dtype_t dtype, int T, int n, const void *x0,
                                        const void *z, const uint8_t *z_mask, uint64_t seed,
                                        const smsq_svgd_opts_t *opts, void *xmap_out, void *logpost_out,
                                        void *particles_out, int32_t *status_out, hipStream_t stream)
{
    if (!model || !dtype_ok(dtype) || T < 1 || n < 1) return SMSQ_ERR_INVALID;
    if (run_layout(dtype, model->desc, 1, T, n).total > kNoallocBytes) return SMSQ_ERR_WORKSPACE;
    void *ws = nullptr;
    smsq_status_t st = scratch_address(&ws);
    if (st != SMSQ_OK) return st;
    st = run_batch_ws(model, dtype, 1, T, n, x0, z, z_mask, seed, opts, xmap_out, logpost_out, particles_out, ws,
                      kNoallocBytes, stream);
    if (st != SMSQ_OK || !status_out) return st;
    hipLaunchKernelGGL(k_status_out, dim3(1), dim3(kWave), 0, stream, (const uint32_t *)ws, status_out);
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

smsq_status_t smsq_get_device_status(const void *ws, smsq_status_t *out)
{
    if (!ws || !out) return SMSQ_ERR_INVALID;
    uint32_t v = 0;
    if (hipMemcpy(&v, ws, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return SMSQ_ERR_HIP;
    *out = (v & STATUS_STALLED) ? SMSQ_ERR_HIP : (v & STATUS_NONFINITE) ? SMSQ_ERR_NONFINITE : SMSQ_OK;
    return SMSQ_OK;
}

smsq_status_t smsq_clear_device_status(void *ws, hipStream_t stream)
{
    if (!ws) return SMSQ_ERR_INVALID;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, status_ptr(ws), 0u, 1);
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

smsq_status_t smsq_batch_plan_create(const smsq_model_t *models, const smsq_svgd_opts_t *opts, int n_models,
                                     const smsq_batch_seq_t *seqs, int count, smsq_batch_plan_t *out)
{
    if (!out) return SMSQ_ERR_INVALID;
    *out = nullptr;
    if (!models || !opts || n_models < 1 || !seqs || count < 1) return SMSQ_ERR_INVALID;
    for (int k = 0; k < n_models; ++k) {
        if (!models[k] || !opts_ok(&opts[k]) || opts[k].step_kernel != SMSQ_STEP_AUTO) return SMSQ_ERR_INVALID;
        if (opts[k].kernel != SMSQ_KERNEL_RBF) return SMSQ_ERR_UNSUPPORTED;  // the plan's step body is RBF
    }
    long lds = 0;
    int T_max = 0, max_n = 0;
    size_t n_parts = 0, n_phi = 0, n_T = 0;
    for (int i = 0; i < count; ++i) {
        const smsq_batch_seq_t &q = seqs[i];
        if (q.model < 0 || q.model >= n_models || q.n < 1 || q.T < 1 || !q.x0 || !q.z || !q.xmap_out ||
            !q.logpost_out || (q.use_proposal != 0 && q.use_proposal != 1))
            return SMSQ_ERR_INVALID;
        const smsq_model_desc_t &d = models[q.model]->desc;
        if (batch_code(d) < 0) return SMSQ_ERR_UNSUPPORTED;
        const MfmaLds L1(q.n, q.n), L2(q.n, 1);
        if (L1.npad > kMaxParticles || L1.total > kLdsLimit - kBatchStaticLds ||
            L2.total > kLdsLimit - kBatchStaticLds)
            return SMSQ_ERR_UNSUPPORTED;
        lds = std::max(lds, std::max(L1.total, L2.total));
        max_n = std::max(max_n, q.n);
        T_max = std::max(T_max, q.T);
        n_parts += (size_t)q.T * q.n * d.d;
        n_phi += (size_t)q.T * q.n;
        n_T += (size_t)q.T;
    }
    if (batch_kernel_attrs() != hipSuccess) return SMSQ_ERR_HIP;
    smsq_batch_plan_s *p = new (std::nothrow) smsq_batch_plan_s;
    if (!p) return SMSQ_ERR_HIP;
    p->count = count;
    p->T_max = T_max;
    p->max_n = max_n;
    p->lds = (size_t)lds;
    // per-step lists, longest processing time first (n^2 L, then sequence index)
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    auto cost = [&](int i) { return (double)seqs[i].n * seqs[i].n * opts[seqs[i].model].n_iter; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    std::vector<int> lists;
    lists.reserve(n_T);
    p->list_off.resize(T_max);
    p->list_cnt.resize(T_max);
    for (int t = 1; t <= T_max; ++t) {
        p->list_off[t - 1] = (int)lists.size();
        for (int i : order)
            if (seqs[i].T >= t) lists.push_back(i);
        p->list_cnt[t - 1] = (int)lists.size() - p->list_off[t - 1];
        p->max_active = std::max(p->max_active, p->list_cnt[t - 1]);
    }
    size_t total = 0;
    hipError_t e = dev_alloc(&p->seqs, (size_t)count, total);
    if (e == hipSuccess) e = dev_alloc(&p->lists, lists.size(), total);
    if (e == hipSuccess) e = dev_alloc(&p->items, (size_t)p->max_active, total);
    if (e == hipSuccess) e = dev_alloc(&p->codes, (size_t)p->max_active, total);
    if (e == hipSuccess) e = dev_alloc(&p->counters, (size_t)T_max, total);
    if (e == hipSuccess) e = dev_alloc(&p->status, (size_t)1, total);
    if (e == hipSuccess) e = dev_alloc(&p->parts, n_parts, total);
    if (e == hipSuccess) e = dev_alloc(&p->phis, n_phi, total);
    if (e == hipSuccess) e = dev_alloc(&p->psis, n_phi, total);
    if (e == hipSuccess) e = dev_alloc(&p->idx, n_T, total);
    if (e != hipSuccess) {
        p->free_all();
        delete p;
        return SMSQ_ERR_HIP;
    }
    p->device_bytes = total;
    p->host.resize(count);
    size_t o_parts = 0, o_phi = 0, o_T = 0;
    for (int i = 0; i < count; ++i) {
        const smsq_batch_seq_t &q = seqs[i];
        const smsq_model_desc_t &d = models[q.model]->desc;
        const smsq_svgd_opts_t &o = opts[q.model];
        SeqDesc &sd = p->host[i];
        std::memset(&sd, 0, sizeof(sd));
        sd.m = make_dev_model<float>(d);
        sd.x0 = (const float *)q.x0;
        sd.z = (const float *)q.z;
        sd.mask = q.z_mask;
        sd.parts = p->parts + o_parts;
        sd.phis = p->phis + o_phi;
        sd.psis = p->psis + o_phi;
        sd.idx = p->idx + o_T;
        sd.xmap = (float *)q.xmap_out;
        sd.logpost = (float *)q.logpost_out;
        sd.n = q.n;
        sd.T = q.T;
        sd.d = d.d;
        sd.code = batch_code(d);
        p->proposal_ok &= batch_family(d.kind);
        sd.n_iter = o.n_iter;
        sd.bw_mode = o.bw_mode;
        sd.trans_mode = o.trans_mode;
        sd.weights = o.weights;
        sd.use_proposal = q.use_proposal;
        sd.step = (float)o.step;
        sd.bw_scale = (float)o.bw_scale;
        sd.seed = q.seed;
        o_parts += (size_t)q.T * q.n * d.d;
        o_phi += (size_t)q.T * q.n;
        o_T += (size_t)q.T;
    }
    e = hipMemcpy(p->seqs, p->host.data(), sizeof(SeqDesc) * count, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->lists, lists.data(), sizeof(int) * lists.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        p->free_all();
        delete p;
        return SMSQ_ERR_HIP;
    }
    *out = p;
    return SMSQ_OK;
}

smsq_status_t smsq_batch_plan_tune(smsq_batch_plan_t p, int steps, hipStream_t stream)
{
    if (!p || steps < 2) return SMSQ_ERR_INVALID;
    const int k = std::min(steps, p->T_max);
    if (k < 2) return SMSQ_OK;
    const std::string key = tune_key(p, k);
    if (!key.empty()) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        const auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            p->waves = it->second.waves;
            p->tuned[0] = it->second.ms[0];
            p->tuned[1] = it->second.ms[1];
            return SMSQ_OK;
        }
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return SMSQ_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SMSQ_ERR_HIP;
    }
    const int shapes[2] = {16, 8};
    smsq_status_t st = SMSQ_OK;
    for (int c = 0; c < 2 && st == SMSQ_OK; ++c) {
        p->waves = shapes[c];
        st = p->reset(stream);
        if (st == SMSQ_OK) st = p->step(1, stream);
        if (st != SMSQ_OK) break;
        if (hipEventRecord(e0, stream) != hipSuccess) { st = SMSQ_ERR_HIP; break; }
        for (int t = 2; t <= k && st == SMSQ_OK; ++t) st = p->step(t, stream);
        if (st != SMSQ_OK) break;
        float ms = 0.f;
        if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = SMSQ_ERR_HIP;
            break;
        }
        p->tuned[c] = ms / (k - 1);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SMSQ_OK) return st;
    p->waves = p->tuned[1] < p->tuned[0] ? 8 : 16;
    if (!key.empty()) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune[key] = TuneRecord{p->waves, {p->tuned[0], p->tuned[1]}};
    }
    return SMSQ_OK;
}

smsq_status_t smsq_batch_run(smsq_batch_plan_t p, int use_graph, hipStream_t stream)
{
    if (!p) return SMSQ_ERR_INVALID;
    if (!use_graph) return p->enqueue(stream);
    if (stream == nullptr) return SMSQ_ERR_INVALID;
    if (!p->exec || p->graph_waves != p->waves || p->graph_mlp != p->mlp) {
        if (p->exec) (void)hipGraphExecDestroy(p->exec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        p->exec = nullptr;
        p->graph = nullptr;
        if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return SMSQ_ERR_HIP;
        const smsq_status_t st = p->enqueue(stream);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(stream, &g);
        if (st != SMSQ_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return st != SMSQ_OK ? st : SMSQ_ERR_HIP;
        }
        p->graph = g;
        if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            p->exec = nullptr;
            return SMSQ_ERR_HIP;
        }
        p->graph_waves = p->waves;
        p->graph_mlp = p->mlp;
    }
    return hipGraphLaunch(p->exec, stream) == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

smsq_status_t smsq_batch_storage(smsq_batch_plan_t p, int seq, void **particles, void **phi, int32_t **psi)
{
    if (!p || seq < 0 || seq >= p->count) return SMSQ_ERR_INVALID;
    if (particles) *particles = p->host[seq].parts;
    if (phi) *phi = p->host[seq].phis;
    if (psi) *psi = p->host[seq].psis;
    return SMSQ_OK;
}

smsq_status_t smsq_batch_plan_info(smsq_batch_plan_t p, smsq_batch_info_t *out)
{
    if (!p || !out) return SMSQ_ERR_INVALID;
    out->count = p->count;
    out->T_max = p->T_max;
    out->waves = p->waves;
    out->grid = p->grid();
    out->lds_bytes = p->lds;
    out->device_bytes = p->device_bytes;
    out->tuned_ms[0] = p->tuned[0];
    out->tuned_ms[1] = p->tuned[1];
    return SMSQ_OK;
}

smsq_status_t smsq_batch_status(smsq_batch_plan_t p, smsq_status_t *out)
{
    if (!p || !out) return SMSQ_ERR_INVALID;
    uint32_t v = 0;
    if (hipMemcpy(&v, p->status, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return SMSQ_ERR_HIP;
    *out = (v & STATUS_STALLED) ? SMSQ_ERR_HIP : (v & STATUS_NONFINITE) ? SMSQ_ERR_NONFINITE : SMSQ_OK;
    return SMSQ_OK;
}

smsq_status_t smsq_batch_plan_destroy(smsq_batch_plan_t p)
{
    if (!p) return SMSQ_ERR_INVALID;
    p->free_all();
    delete p;
    return SMSQ_OK;
}

smsq_status_t smsq_init_mlp_create(uint64_t seed, int max_batch, smsq_init_mlp_t *out)
{
    if (!out) return SMSQ_ERR_INVALID;
    *out = nullptr;
    if (max_batch < 1 || max_batch > (1 << 20)) return SMSQ_ERR_INVALID;
    smsq_init_mlp_s *m = new (std::nothrow) smsq_init_mlp_s;
    if (!m) return SMSQ_ERR_HIP;
    m->max_batch = max_batch;
    const size_t B = (size_t)max_batch, H = kInitHidden;
    size_t t = 0;
    hipError_t e = zero_alloc_bytes((void **)&m->P, kInitParams * 4, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->G, kInitParams * 4, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->Mo, kInitParams * 4, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->Ve, kInitParams * 4, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->w1b, H * kInitFeat * 2, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->w2b, H * H * 2, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->w3b, kInitOutPad * H * 2, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->F, B * kInitFeat * 4, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->Fb, B * kInitFeat * 2, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->anc, B * 8 * 4, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->scl, B * 8 * 4, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->pre1, B * H * 4, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->pre2, B * H * 4, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->h1, B * H * 2, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->h2, B * H * 2, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->out, B * kInitOut * 4, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->dout, B * kInitOut * 4, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->doutb, B * kInitOut * 2, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->d2, B * H * 4, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->d1, B * H * 4, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->d2b, B * H * 2, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->d1b, B * H * 2, t);
    if (e == hipSuccess) e = zero_alloc_bytes((void **)&m->lossv, B * 4, t);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_init_he, dim3((kInitParams + 255) / 256), dim3(256), 0, nullptr, m->P, seed);
        hipLaunchKernelGGL(k_init_weights_bf16, dim3((kInitParams + 255) / 256), dim3(256), 0, nullptr, m->P,
                           m->w1b, m->w2b, m->w3b);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    if (e != hipSuccess) {
        m->free_all();
        delete m;
        return SMSQ_ERR_HIP;
    }
    m->bytes = t;
    *out = m;
    return SMSQ_OK;
}

smsq_status_t smsq_init_mlp_destroy(smsq_init_mlp_t m)
{
    if (!m) return SMSQ_ERR_INVALID;
    m->free_all();
    delete m;
    return SMSQ_OK;
}

smsq_status_t smsq_init_mlp_params(smsq_init_mlp_t m, float **params, float **grads, size_t *count)
{
    if (!m) return SMSQ_ERR_INVALID;
    if (params) *params = m->P;
    if (grads) *grads = m->G;
    if (count) *count = (size_t)kInitParams;
    return SMSQ_OK;
}

smsq_status_t smsq_init_mlp_sync(smsq_init_mlp_t m, hipStream_t s)
{
    if (!m) return SMSQ_ERR_INVALID;
    hipLaunchKernelGGL(k_init_weights_bf16, dim3((kInitParams + 255) / 256), dim3(256), 0, s, m->P, m->w1b, m->w2b,
                       m->w3b);
    hipLaunchKernelGGL(k_fill_f32, dim3((kInitParams + 255) / 256), dim3(256), 0, s, m->Mo, 0.f, kInitParams);
    hipLaunchKernelGGL(k_fill_f32, dim3((kInitParams + 255) / 256), dim3(256), 0, s, m->Ve, 0.f, kInitParams);
    m->adam_t = 0;
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

smsq_status_t smsq_init_set_create(const smsq_model_t *models, int n_models, const smsq_init_example_t *ex,
                                   int count, smsq_init_set_t *out)
{
    if (!out) return SMSQ_ERR_INVALID;
    *out = nullptr;
    if (!models || n_models < 1 || !ex || count < 1) return SMSQ_ERR_INVALID;
    std::vector<InitExample> h(count);
    int max_n = 0;
    for (int i = 0; i < count; ++i) {
        const smsq_init_example_t &q = ex[i];
        if (q.model < 0 || q.model >= n_models || !models[q.model] || q.t < 2 || q.n < 1 || q.n_prev < 1 ||
            !q.x_prev || !q.phi_prev || !q.z || !q.particles)
            return SMSQ_ERR_INVALID;
        const smsq_model_desc_t &d = models[q.model]->desc;
        if (!batch_family(d.kind)) return SMSQ_ERR_UNSUPPORTED;
        InitExample &x = h[i];
        std::memset(&x, 0, sizeof(x));
        x.m = make_dev_model<float>(d);
        x.xprev = (const float *)q.x_prev;
        x.phiprev = (const float *)q.phi_prev;
        x.z = (const float *)q.z;
        x.mask = q.z_mask;
        x.target = (float *)q.particles;
        x.np = q.n_prev;
        x.n = q.n;
        x.t = q.t;
        x.code = d.kind;
        x.seq = q.seq;
        x.seed = q.seed;
        max_n = std::max(max_n, q.n);
    }
    smsq_init_set_s *st = new (std::nothrow) smsq_init_set_s;
    if (!st) return SMSQ_ERR_HIP;
    st->count = count;
    st->max_n = max_n;
    if (hipMalloc((void **)&st->ex, sizeof(InitExample) * count) != hipSuccess ||
        hipMemcpy(st->ex, h.data(), sizeof(InitExample) * count, hipMemcpyHostToDevice) != hipSuccess) {
        if (st->ex) (void)hipFree(st->ex);
        delete st;
        return SMSQ_ERR_HIP;
    }
    *out = st;
    return SMSQ_OK;
}

smsq_status_t smsq_init_set_destroy(smsq_init_set_t st)
{
    if (!st) return SMSQ_ERR_INVALID;
    if (st->ex) (void)hipFree(st->ex);
    delete st;
    return SMSQ_OK;
}

namespace {
bool range_ok(smsq_init_mlp_s *m, smsq_init_set_s *st, int first, int count)
{
    return m && st && first >= 0 && count >= 1 && first + count <= st->count && count <= m->max_batch;
}
} // namespace

smsq_status_t smsq_init_features(smsq_init_mlp_t m, smsq_init_set_t st, int first, int count, void *features,
                                 void *anchors, void *scales, hipStream_t s)
{
    if (!range_ok(m, st, first, count)) return SMSQ_ERR_INVALID;
    mlp_features(m, st->ex + first, count, s);
    if (features && hipMemcpyAsync(features, m->F, (size_t)count * kInitFeat * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return SMSQ_ERR_HIP;
    if (anchors && hipMemcpyAsync(anchors, m->anc, (size_t)count * 8 * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return SMSQ_ERR_HIP;
    if (scales && hipMemcpyAsync(scales, m->scl, (size_t)count * 8 * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return SMSQ_ERR_HIP;
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

smsq_status_t smsq_init_mlp_forward(smsq_init_mlp_t m, int batch, const void *features, void *out, hipStream_t s)
{
    if (!m || batch < 1 || batch > m->max_batch || !features || !out) return SMSQ_ERR_INVALID;
    hipLaunchKernelGGL(k_to_bf16, dim3((batch * kInitFeat + 255) / 256), dim3(256), 0, s, (const float *)features,
                       m->Fb, (long)batch * kInitFeat);
    mlp_forward(m, batch, s);
    if (hipMemcpyAsync(out, m->out, (size_t)batch * kInitOut * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return SMSQ_ERR_HIP;
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

smsq_status_t smsq_init_mlp_backward(smsq_init_mlp_t m, int batch, const void *dout, hipStream_t s)
{
    if (!m || batch < 1 || batch > m->max_batch || !dout) return SMSQ_ERR_INVALID;
    if (hipMemcpyAsync(m->dout, dout, (size_t)batch * kInitOut * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return SMSQ_ERR_HIP;
    mlp_backward(m, batch, s);
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

smsq_status_t smsq_init_mixture_nll(smsq_init_set_t st, int first, int count, const void *out, const void *anchors,
                                    const void *scales, double gscale, void *loss, void *dout, hipStream_t s)
{
    if (!st || first < 0 || count < 1 || first + count > st->count || !out || !anchors || !scales || !loss || !dout)
        return SMSQ_ERR_INVALID;
    hipLaunchKernelGGL(k_mix_nll, dim3(count), dim3(kWave), 0, s, st->ex + first, count, (const float *)out,
                       (const float *)anchors, (const float *)scales, (float *)dout, (float *)loss, (float)gscale);
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

smsq_status_t smsq_init_mlp_train_step(smsq_init_mlp_t m, smsq_init_set_t st, int first, int count, double lr,
                                       void *loss_out, hipStream_t s)
{
    if (!range_ok(m, st, first, count) || !(lr > 0.0)) return SMSQ_ERR_INVALID;
    const InitExample *ex = st->ex + first;
    mlp_features(m, ex, count, s);
    mlp_forward(m, count, s);
    hipLaunchKernelGGL(k_mix_nll, dim3(count), dim3(kWave), 0, s, ex, count, m->out, m->anc, m->scl, m->dout,
                       m->lossv, 1.f / (float)count);
    mlp_backward(m, count, s);
    m->adam_t += 1;
    // Adam constants as FP32 values; their bias corrections in FP64
    const float b1 = 0.9f, b2 = 0.999f;
    const double c1 = 1.0 / (1.0 - std::pow((double)b1, m->adam_t));
    const double c2 = 1.0 / (1.0 - std::pow((double)b2, m->adam_t));
    hipLaunchKernelGGL(k_adam, dim3((kInitParams + 255) / 256), dim3(256), 0, s, m->P, m->G, m->Mo, m->Ve,
                       kInitParams, (float)lr, b1, b2, 1e-8f, (float)c1, (float)c2, m->w1b, m->w2b, m->w3b);
    if (loss_out) hipLaunchKernelGGL(k_mean_f32, dim3(1), dim3(kWave), 0, s, m->lossv, count, (float *)loss_out);
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

smsq_status_t smsq_init_mlp_sample(smsq_init_mlp_t m, smsq_init_set_t st, int first, int count, int32_t *used,
                                   hipStream_t s)
{
    if (!range_ok(m, st, first, count)) return SMSQ_ERR_INVALID;
    return init_propose(m, st->ex + first, count, st->max_n, used, s);
}

smsq_status_t smsq_batch_plan_set_init(smsq_batch_plan_t p, smsq_init_mlp_t m)
{
    if (!p) return SMSQ_ERR_INVALID;
    if (m && !p->proposal_ok) return SMSQ_ERR_UNSUPPORTED;   // the proposal's features cover four families
    if (m && m->max_batch < p->max_active) return SMSQ_ERR_INVALID;
    if (m && !p->init_ex) {
        size_t total = 0;
        if (dev_alloc(&p->init_ex, (size_t)p->max_active, total) != hipSuccess ||
            dev_alloc(&p->init_used, (size_t)p->max_active, total) != hipSuccess)
            return SMSQ_ERR_HIP;
        p->device_bytes += total;
    }
    p->mlp = m;
    return SMSQ_OK;
}

const char *smsq_status_string(smsq_status_t s)
{
    switch (s) {
    case SMSQ_OK: return "ok";
    case SMSQ_ERR_INVALID: return "invalid argument";
    case SMSQ_ERR_UNSUPPORTED: return "unsupported shape";
    case SMSQ_ERR_HIP: return "HIP runtime error";
    case SMSQ_ERR_NONFINITE: return "non-finite value on device";
    case SMSQ_ERR_WORKSPACE: return "workspace missing or too small";
    }
    return "unknown status";
}

} // extern "C"
