// C ABI of the Stein-MAP-Seq hot path (declarations and contracts in
// include/smsq.h).  Host code: argument validation, workspace layout, launch
// configuration and dispatch to the templated kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "smsq.h"
#include "smsq_kernels.hpp"
#include "smsq_mfma.hpp"

#include <cstdlib>

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
    for (int c = 0; c < d->d && c < 8; ++c)
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
    for (int c = 0; c < 8; ++c) {
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
    if (d.kind == SMSQ_MODEL_ARM7)
        for (int i = 0; i < 7; ++i) {
            m.aux[i] = (T)std::cos(d.params[8 + i]);
            m.aux[7 + i] = (T)std::sin(d.params[8 + i]);
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

template <typename KernelFn> hipError_t allow_big_lds(KernelFn fn)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
}

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

// The FP32 matrix-core kernel takes sequences of up to 1024 particles whose
// state fits LDS; SMSQ_STEP_KERNEL=valu selects the vector-ALU kernel instead.
bool use_mfma(int n, int n_prev)
{
    const char *e = std::getenv("SMSQ_STEP_KERNEL");
    if (e && std::strcmp(e, "valu") == 0) return false;
    const MfmaLds L(n, n_prev);
    return L.npad <= kMaxParticles && L.total <= kLdsLimit;
}

template <int KIND, int D>
smsq_status_t launch_mfma_kd(const StepArgs<float> &a, int batch, hipStream_t s)
{
    auto fn = &k_step_mfma<KIND, D>;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [&] { attr_err = allow_big_lds(fn); });
    if (attr_err != hipSuccess) return SMSQ_ERR_HIP;
    const MfmaLds L(a.n, a.n_prev);
    hipLaunchKernelGGL(fn, dim3(batch), dim3(L.nwaves * kWave), (size_t)L.total, s, a);
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
}

template <typename T>
smsq_status_t launch_step(const smsq_model_desc_t &d, const StepArgs<T> &a, int batch, hipStream_t s);

template <>
smsq_status_t launch_step<float>(const smsq_model_desc_t &d, const StepArgs<float> &a, int batch, hipStream_t s)
{
    if (use_mfma(a.n, a.n_prev)) {
        switch (d.kind) {
        case SMSQ_MODEL_GROWTH1D: return launch_mfma_kd<GROWTH1D, 1>(a, batch, s);
        case SMSQ_MODEL_RANGE2D: return launch_mfma_kd<RANGE2D, 2>(a, batch, s);
        case SMSQ_MODEL_CV4D: return launch_mfma_kd<CV4D, 4>(a, batch, s);
        case SMSQ_MODEL_ARM7: return launch_mfma_kd<ARM7, 7>(a, batch, s);
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
smsq_status_t launch_step<double>(const smsq_model_desc_t &d, const StepArgs<double> &a, int batch, hipStream_t s)
{
    switch (d.kind) {
    case SMSQ_MODEL_GROWTH1D: return launch_step_kd<double, GROWTH1D, 1>(a, batch, s);
    case SMSQ_MODEL_RANGE2D: return launch_step_kd<double, RANGE2D, 2>(a, batch, s);
    case SMSQ_MODEL_CV4D: return launch_step_kd<double, CV4D, 4>(a, batch, s);
    case SMSQ_MODEL_ARM7: return launch_step_kd<double, ARM7, 7>(a, batch, s);
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

bool opts_ok(const smsq_svgd_opts_t *o)
{
    return o && o->n_iter >= 0 && std::isfinite(o->step) && finite_pos(o->bw_scale) &&
           (o->bw_mode == 0 || o->bw_mode == 1) && (o->trans_mode == 0 || o->trans_mode == 1);
}

uint32_t *status_ptr(void *ws) { return reinterpret_cast<uint32_t *>(ws); }

// Generic batched step launch (typed).
template <typename T>
smsq_status_t step_typed(const smsq_model_desc_t &d, int batch, int t, int n_prev, const void *x_prev,
                         long x_prev_stride, const void *log_w, long log_w_stride, const void *phi_prev,
                         long phi_prev_stride, const void *z, long z_stride, const uint8_t *mask,
                         long mask_stride, int n, void *x, long x_stride, int init_given, uint64_t seed,
                         uint32_t seq_offset, const smsq_svgd_opts_t *opts, bool do_svgd, bool do_viterbi,
                         void *phi, long phi_stride, int32_t *psi, long psi_stride, uint8_t *flags,
                         long flags_stride, double tie_tol, void *h_out, long h_stride, void *ws,
                         hipStream_t s)
{
    StepArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.m = make_dev_model<T>(d);
    a.x_prev = (const T *)x_prev; a.x_prev_stride = x_prev_stride;
    a.log_w = (const T *)log_w; a.log_w_stride = log_w_stride;
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
    a.init_given = init_given;
    a.do_svgd = do_svgd ? 1 : 0;
    a.do_viterbi = do_viterbi ? 1 : 0;
    a.step = (T)(opts ? opts->step : 0.0);
    a.bw_scale = (T)(opts ? opts->bw_scale : 1.0);
    a.tie_tol = (T)tie_tol;
    a.seed = seed; a.seq_offset = seq_offset;
    return launch_step<T>(d, a, batch, s);
}

smsq_status_t step_dispatch(smsq_dtype_t dt, const smsq_model_desc_t &d, int batch, int t, int n_prev,
                            const void *x_prev, long x_prev_stride, const void *log_w, long log_w_stride,
                            const void *phi_prev, long phi_prev_stride, const void *z, long z_stride,
                            const uint8_t *mask, long mask_stride, int n, void *x, long x_stride,
                            int init_given, uint64_t seed, uint32_t seq_offset, const smsq_svgd_opts_t *opts,
                            bool do_svgd, bool do_viterbi, void *phi, long phi_stride, int32_t *psi,
                            long psi_stride, uint8_t *flags, long flags_stride, double tie_tol, void *h_out,
                            long h_stride, void *ws, hipStream_t s)
{
    if (dt == SMSQ_F64)
        return step_typed<double>(d, batch, t, n_prev, x_prev, x_prev_stride, log_w, log_w_stride, phi_prev,
                                  phi_prev_stride, z, z_stride, mask, mask_stride, n, x, x_stride, init_given,
                                  seed, seq_offset, opts, do_svgd, do_viterbi, phi, phi_stride, psi, psi_stride,
                                  flags, flags_stride, tie_tol, h_out, h_stride, ws, s);
    return step_typed<float>(d, batch, t, n_prev, x_prev, x_prev_stride, log_w, log_w_stride, phi_prev,
                             phi_prev_stride, z, z_stride, mask, mask_stride, n, x, x_stride, init_given, seed,
                             seq_offset, opts, do_svgd, do_viterbi, phi, phi_stride, psi, psi_stride, flags,
                             flags_stride, tie_tol, h_out, h_stride, ws, s);
}

struct RunLayout {
    size_t parts, psi, phi, idx, total;
};

RunLayout run_layout(smsq_dtype_t dt, int batch, int T, int n, int d)
{
    RunLayout L;
    size_t o = kHeader;
    const size_t es = elem_size(dt);
    L.parts = o; o += align256((size_t)batch * T * n * d * es);
    L.psi = o; o += align256((size_t)batch * T * n * sizeof(int32_t));
    L.phi = o; o += align256((size_t)2 * batch * n * es);
    L.idx = o; o += align256((size_t)batch * T * sizeof(int32_t));
    L.total = o;
    return L;
}

bool dtype_ok(smsq_dtype_t dt) { return dt == SMSQ_F32 || dt == SMSQ_F64; }

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
    *bytes = run_layout(dtype, batch, T, n, model->desc.d).total;
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
        const int rows_per_block = 4;
        const dim3 grid((n + rows_per_block - 1) / rows_per_block), block(rows_per_block * kWave);
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
    if (!step_shape_ok(dtype, n, n_prev, model->desc.d)) return SMSQ_ERR_UNSUPPORTED;
    // particle mode: the step kernel with no SVGD iteration and the given particles
    return step_dispatch(dtype, model->desc, 1, t, n_prev, x_prev, 0, nullptr, 0, phi_prev, 0, z_t, 0, z_mask,
                         0, n, const_cast<void *>(x), 0, 1, 0, 0, nullptr, false, true, phi, 0, psi, 0,
                         tie_flags, 0, tie_tol, nullptr, 0, ws, stream);
}

smsq_status_t smsq_backtrack(smsq_dtype_t dtype, int batch, int T, int n, int d, const int32_t *psi,
                             const void *phi_T, int32_t *idx_out, void *logpost_out, const void *particles,
                             const void *x0, void *xmap_out, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!dtype_ok(dtype) || batch < 1 || T < 1 || n < 1 || !psi || !phi_T || !idx_out || !logpost_out)
        return SMSQ_ERR_INVALID;
    const bool gather = particles && x0 && xmap_out;
    if (gather && (d < 1 || d > 8)) return SMSQ_ERR_INVALID;
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
    if (!model || !dtype_ok(dtype) || batch < 1 || T < 1 || n < 1 || !x0 || !z || !opts_ok(opts) || !xmap_out ||
        !logpost_out)
        return SMSQ_ERR_INVALID;
    const smsq_model_desc_t &d = model->desc;
    const RunLayout L = run_layout(dtype, batch, T, n, d.d);
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
            psi + (size_t)(t - 1) * n, (long)T * n, nullptr, 0, 0.0, nullptr, 0, ws, stream);
        if (st != SMSQ_OK) return st;
    }
    return smsq_backtrack(dtype, batch, T, n, d.d, psi, phi_buf[T & 1], idx, logpost_out, parts, x0, xmap_out, ws,
                          ws_bytes, stream);
}

smsq_status_t smsq_run_sequence(smsq_model_t model, smsq_dtype_t dtype, int T, int n, const void *x0,
                                const void *z, const uint8_t *z_mask, uint64_t seed, const smsq_svgd_opts_t *opts,
                                void *xmap_out, void *logpost_out, void *particles_out, void *ws, size_t ws_bytes,
                                hipStream_t stream)
{
    return smsq_run_batch(model, dtype, 1, T, n, x0, z, z_mask, seed, opts, xmap_out, logpost_out, particles_out,
                          ws, ws_bytes, stream);
}

smsq_status_t smsq_get_device_status(const void *ws, smsq_status_t *out)
{
    if (!ws || !out) return SMSQ_ERR_INVALID;
    uint32_t v = 0;
    if (hipMemcpy(&v, ws, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return SMSQ_ERR_HIP;
    *out = (v & STATUS_NONFINITE) ? SMSQ_ERR_NONFINITE : SMSQ_OK;
    return SMSQ_OK;
}

smsq_status_t smsq_clear_device_status(void *ws, hipStream_t stream)
{
    if (!ws) return SMSQ_ERR_INVALID;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, status_ptr(ws), 0u, 1);
    return hipGetLastError() == hipSuccess ? SMSQ_OK : SMSQ_ERR_HIP;
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
