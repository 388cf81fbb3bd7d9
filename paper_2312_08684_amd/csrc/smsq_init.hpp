// Learned particle initialisation: a small MLP maps a summary of the
// previous step's particle set and the new observation to a K-component
// diagonal Gaussian mixture, from which the N initial particles of the step
// are drawn (the predictive initialisation stays the fallback).  The
// proposal is trained on converged particle sets the method produces, by the
// mixture negative log-likelihood.  GEMMs take BF16 operands and accumulate
// in FP32 on the matrix cores (v_mfma_f32_16x16x16bf16_1k).
//
// Features (64, zero padded), with a = f_t(x_{t-1}^{best}), best the lowest
// argmax of the previous forward-recursion scores, M_j = f_t(x_{t-1}^j) and
// s = sqrt(q):
//   [0..3]   family one-hot
//   [4]      ln(n) / 7
//   [5..11]  (mean_j M_j - a) / s
//   [12..18] ln(var_j M_j / s^2 + 1e-6) / 8
//   [19..25] asinh(s * grad_x log p(z_t | a)) / 4
//   [26]     asinh(log p(z_t | a)) / 8
//   [27..63] zero
// (entries k >= d of each per-dimension block are zero).  No feature holds
// the absolute position: the mixture is placed relative to a.
// Outputs (120 = 8 x 15): component c has logit o[15c], mean offsets
// o[15c + 1 + k] and log-scales o[15c + 8 + k]: mean a + s mu, standard
// deviation s exp(clamp(rho, -7, 3)) per dimension k < d.
#pragma once

#include "smsq_batch.hpp"

namespace smsq {

constexpr int kInitFeat = 64;
constexpr int kInitHidden = 256;
constexpr int kInitK = 8;
constexpr int kInitComp = 15;                    // logit + 7 means + 7 log-scales
constexpr int kInitOut = kInitK * kInitComp;     // 120
constexpr int kInitOutPad = 128;
constexpr float kRhoMin = -7.f, kRhoMax = 3.f;
// flattened FP32 parameters: W1 [256][64], b1, W2 [256][256], b2, W3 [120][256], b3
constexpr long kOffW1 = 0;
constexpr long kOffB1 = kOffW1 + (long)kInitHidden * kInitFeat;
constexpr long kOffW2 = kOffB1 + kInitHidden;
constexpr long kOffB2 = kOffW2 + (long)kInitHidden * kInitHidden;
constexpr long kOffW3 = kOffB2 + kInitHidden;
constexpr long kOffB3 = kOffW3 + (long)kInitOut * kInitHidden;
constexpr long kInitParams = kOffB3 + kInitOut;  // 113,272

typedef short bf16x4 __attribute__((ext_vector_type(4)));

// round to nearest even; NaN stays NaN
__host__ __device__ inline uint16_t to_bf16(float f)
{
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__host__ __device__ inline float from_bf16(uint16_t h)
{
    const uint32_t u = (uint32_t)h << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// One example of the proposal: a sequence step (training: `target` holds the
// converged particles; sampling: the initial particles are written there).
struct InitExample {
    DevModel<float> m;
    const float *xprev;     // [np][d]
    const float *phiprev;   // [np] or null (all equal)
    const float *z;         // [obs_dim]
    const uint8_t *mask;    // [n_obs] or null
    float *target;          // [n][d]
    int np, n, t, code, seq;
    uint64_t seed;
};

// Features of examples [0, count): one wave each.  Also the anchor a and
// scale s per example ([8] each).
template <int KIND, int D>
__device__ void init_features_one(const InitExample &e, float *F, uint16_t *Fb, float *anc, float *scl)
{
    using Fm = Family<float, KIND, D>;
    const int lane = threadIdx.x & 63;
    // best previous particle: lowest index among the maxima
    ArgBest<float> ab{-__builtin_huge_valf(), -__builtin_huge_valf(), 0x7fffffff};
    for (int j = lane; j < e.np; j += kWave) {
        const float v = e.phiprev ? e.phiprev[j] : 0.f;
        if (j == lane) { ab.best = v; ab.arg = j; }
        else argbest_push(ab, v, j);
    }
    ab = wave_argbest(ab);
    const int best = ab.arg < e.np ? ab.arg : 0;
    float a[D], xb[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xb[k] = e.xprev[(long)best * D + k];
    Fm::mean(e.m, e.t, xb, a);
    // moments of the propagated set (two passes for the variance)
    float mu[D], var[D];
#pragma unroll
    for (int k = 0; k < D; ++k) mu[k] = 0.f;
    for (int j = lane; j < e.np; j += kWave) {
        float x[D], mj[D];
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = e.xprev[(long)j * D + k];
        Fm::mean(e.m, e.t, x, mj);
#pragma unroll
        for (int k = 0; k < D; ++k) mu[k] += mj[k];
    }
#pragma unroll
    for (int k = 0; k < D; ++k) mu[k] = wave_sum(mu[k]) / (float)e.np;
#pragma unroll
    for (int k = 0; k < D; ++k) var[k] = 0.f;
    for (int j = lane; j < e.np; j += kWave) {
        float x[D], mj[D];
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = e.xprev[(long)j * D + k];
        Fm::mean(e.m, e.t, x, mj);
#pragma unroll
        for (int k = 0; k < D; ++k) var[k] += (mj[k] - mu[k]) * (mj[k] - mu[k]);
    }
#pragma unroll
    for (int k = 0; k < D; ++k) var[k] = wave_sum(var[k]) / (float)e.np;
    float g[D];
    Fm::grad(e.m, e.z, e.mask, a, g);
    const float ll = Fm::loglik(e.m, e.z, e.mask, a);
    // lane f writes feature f; none holds the absolute position (offsets
    // from the anchor, spreads and the likelihood around it only)
    float v = 0.f;
    const int f = lane;
    if (f < 4) v = f == KIND ? 1.f : 0.f;
    else if (f == 4) v = logf((float)e.n) / 7.f;
    else if (f == 26) v = asinhf(ll) / 8.f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const float s = e.m.sqrt_q[k];
        if (f == 5 + k) v = (mu[k] - a[k]) / s;
        if (f == 12 + k) v = logf(var[k] / (s * s) + 1e-6f) / 8.f;
        if (f == 19 + k) v = asinhf(s * g[k]) / 4.f;
    }
    F[f] = v;
    Fb[f] = to_bf16(v);
    if (lane < 8) {
        float av = 0.f, sv = 1.f;
#pragma unroll
        for (int k = 0; k < D; ++k)
            if (lane == k) { av = a[k]; sv = e.m.sqrt_q[k]; }
        anc[lane] = av;
        scl[lane] = sv;
    }
}

__global__ __launch_bounds__(64) void k_init_features(const InitExample *__restrict__ ex, int count,
                                                      float *F, uint16_t *Fb, float *anc, float *scl)
{
    const int e = blockIdx.x;
    if (e >= count) return;
    const InitExample &x = ex[e];
    float *f = F + (long)e * kInitFeat;
    uint16_t *fb = Fb + (long)e * kInitFeat;
    switch (x.code) {
    case GROWTH1D: init_features_one<GROWTH1D, 1>(x, f, fb, anc + e * 8, scl + e * 8); break;
    case RANGE2D: init_features_one<RANGE2D, 2>(x, f, fb, anc + e * 8, scl + e * 8); break;
    case CV4D: init_features_one<CV4D, 4>(x, f, fb, anc + e * 8, scl + e * 8); break;
    default: init_features_one<ARM7, 7>(x, f, fb, anc + e * 8, scl + e * 8); break;
    }
}

// C[m][n] = sum_k A(m, k) B(k, n) with BF16 operands read through element
// strides (A(m,k) = A[m sam + k sak], B(k,n) = B[k sbk + n sbn]), FP32
// accumulation, one 16x16 tile per wave.  Epilogue modes:
//   0 hidden forward: pre = acc + bias -> C (FP32), relu(pre) -> Cb (BF16)
//   1 output forward: acc + bias -> C
//   2 data gradient through a ReLU: acc * (pre[m][n] > 0) -> C, Cb
//   3 weight gradient: acc -> C
// Operand layout of v_mfma_f32_16x16x16bf16_1k: lane l gives A[l % 16][4 (l /
// 16) + j] and B[4 (l / 16) + j][l % 16], j = 0..3; result register r of lane
// l is C[4 (l / 16) + r][l % 16].
__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const uint16_t *__restrict__ A, long sam,
                                                   long sak, const uint16_t *__restrict__ B, long sbk, long sbn,
                                                   float *C, long ldc, uint16_t *Cb, long ldcb,
                                                   const float *__restrict__ bias, const float *__restrict__ pre,
                                                   long ldpre, int mode)
{
    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int tn = (N + 15) / 16;
    const int tm = tile / tn, tc = tile % tn;
    if (tm * 16 >= M) return;
    const int g = lane >> 4, col = lane & 15;
    const int am = tm * 16 + col;   // A row of this lane
    const int bn = tc * 16 + col;   // B column of this lane
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x4 av, bv;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = k0 + 4 * g + j;
            av[j] = (am < M && k < K) ? (short)A[(long)am * sam + (long)k * sak] : (short)0;
            bv[j] = (bn < N && k < K) ? (short)B[(long)k * sbk + (long)bn * sbn] : (short)0;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int m = tm * 16 + 4 * g + r, n = tc * 16 + col;
        if (m >= M || n >= N) continue;
        float v = acc[r];
        if (mode == 0) {
            v += bias[n];
            C[(long)m * ldc + n] = v;
            Cb[(long)m * ldcb + n] = to_bf16(v > 0.f ? v : 0.f);
        } else if (mode == 1) {
            C[(long)m * ldc + n] = v + bias[n];
        } else if (mode == 2) {
            v = pre[(long)m * ldpre + n] > 0.f ? v : 0.f;
            C[(long)m * ldc + n] = v;
            Cb[(long)m * ldcb + n] = to_bf16(v);
        } else {
            C[(long)m * ldc + n] = v;
        }
    }
}

// db[n] = sum_m dY[m][n] (FP32)
__global__ void k_colsum(int M, int N, const float *__restrict__ dY, long ld, float *db)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += dY[(long)m * ld + n];
    db[n] = s;
}

__global__ void k_to_bf16(const float *__restrict__ src, uint16_t *dst, long count)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = to_bf16(src[i]);
}

// Mixture NLL of each example's target particles and its gradient with
// respect to the 120 outputs (scaled by gscale).  One wave per example.
__global__ __launch_bounds__(64) void k_mix_nll(const InitExample *__restrict__ ex, int count,
                                                const float *__restrict__ out, const float *__restrict__ anc,
                                                const float *__restrict__ scl, float *dout, float *loss,
                                                float gscale)
{
    const int e = blockIdx.x;
    if (e >= count) return;
    const int lane = threadIdx.x;
    const InitExample &x = ex[e];
    const int d = x.m.d, n = x.n;
    const float *o = out + (long)e * kInitOut;
    float a[7], s[7], pl[kInitK];
    float mean[kInitK][7], isd[kInitK][7], lsd[kInitK][7];  // mean, 1 / sd, log sd
    bool rin[kInitK][7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        a[k] = anc[e * 8 + k];
        s[k] = scl[e * 8 + k];
    }
    float lmax = -__builtin_huge_valf();
#pragma unroll
    for (int c = 0; c < kInitK; ++c) lmax = fmaxf(lmax, o[c * kInitComp]);
    float lse = 0.f;
#pragma unroll
    for (int c = 0; c < kInitK; ++c) lse += expf(o[c * kInitComp] - lmax);
    lse = lmax + logf(lse);
    float pc[kInitK];
#pragma unroll
    for (int c = 0; c < kInitK; ++c) {
        pl[c] = o[c * kInitComp] - lse;  // log pi_c
        pc[c] = expf(pl[c]);
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            const float r = o[c * kInitComp + 8 + k];
            rin[c][k] = r >= kRhoMin && r <= kRhoMax;
            const float rc = fminf(fmaxf(r, kRhoMin), kRhoMax);
            mean[c][k] = a[k] + s[k] * o[c * kInitComp + 1 + k];
            isd[c][k] = 1.f / (s[k] * expf(rc));
            lsd[c][k] = logf(s[k]) + rc;
        }
    }
    float gl[kInitK], gm[kInitK][7], gr[kInitK][7];
#pragma unroll
    for (int c = 0; c < kInitK; ++c) {
        gl[c] = 0.f;
#pragma unroll
        for (int k = 0; k < 7; ++k) gm[c][k] = gr[c][k] = 0.f;
    }
    float lsum = 0.f;
    const float hl2pi = 0.91893853320467274178f;
    for (int i = lane; i < n; i += kWave) {
        float xi[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) xi[k] = k < d ? x.target[(long)i * d + k] : 0.f;
        float lc[kInitK];
        float mx = -__builtin_huge_valf();
#pragma unroll
        for (int c = 0; c < kInitK; ++c) {
            float v = pl[c];
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                if (k < d) {
                    const float u = (xi[k] - mean[c][k]) * isd[c][k];
                    v += -0.5f * u * u - lsd[c][k] - hl2pi;
                }
            }
            lc[c] = v;
            mx = fmaxf(mx, v);
        }
        float se = 0.f;
#pragma unroll
        for (int c = 0; c < kInitK; ++c) se += expf(lc[c] - mx);
        const float lse_i = mx + logf(se);
        lsum += -lse_i;
#pragma unroll
        for (int c = 0; c < kInitK; ++c) {
            const float r = expf(lc[c] - lse_i);  // responsibility
            gl[c] += -(r - pc[c]);
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                if (k < d) {
                    const float u = (xi[k] - mean[c][k]) * isd[c][k];
                    gm[c][k] += -r * u * isd[c][k] * s[k];
                    gr[c][k] += -r * (u * u - 1.f);
                }
            }
        }
    }
    lsum = wave_sum(lsum);
    const float w = gscale / (float)n;
    float *go = dout + (long)e * kInitOut;
#pragma unroll
    for (int c = 0; c < kInitK; ++c) {
        const float v = wave_sum(gl[c]);
        if (lane == 0) go[c * kInitComp] = v * w;
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            const float vm = wave_sum(gm[c][k]);
            const float vr = wave_sum(gr[c][k]);
            if (lane == 0) {
                go[c * kInitComp + 1 + k] = vm * w;
                go[c * kInitComp + 8 + k] = rin[c][k] ? vr * w : 0.f;
            }
        }
    }
    if (lane == 0) loss[e] = lsum / (float)n;
}

// Draws each example's n particles from its mixture into `target`:
// component from one uniform by the cumulative weights, standard normals by
// Box-Muller, uniforms from Philox4x32-10 keyed by the example seed with
// counter (i, t, seq, 2 + b), b = 0, 1, 2.  Non-finite outputs: used[e] = 0
// and nothing is written (the predictive initialisation applies).
template <int D>
__device__ void mix_sample_one(const InitExample &x, int i, const float *o, const float *anc, const float *scl)
{
    float lmax = -__builtin_huge_valf();
    for (int c = 0; c < kInitK; ++c) lmax = fmaxf(lmax, o[c * kInitComp]);
    float w[kInitK], tot = 0.f;
    for (int c = 0; c < kInitK; ++c) {
        w[c] = expf(o[c * kInitComp] - lmax);
        tot += w[c];
    }
    const uint32_t k0 = (uint32_t)x.seed, k1 = (uint32_t)(x.seed >> 32);
    double u[12];
    for (int b = 0; b < 3; ++b) {
        const U4 r = philox4x32_10(U4{(uint32_t)i, (uint32_t)x.t, (uint32_t)x.seq, 2u + (uint32_t)b}, k0, k1);
        u[4 * b + 0] = ((double)r.x + 0.5) * (1.0 / 4294967296.0);
        u[4 * b + 1] = ((double)r.y + 0.5) * (1.0 / 4294967296.0);
        u[4 * b + 2] = ((double)r.z + 0.5) * (1.0 / 4294967296.0);
        u[4 * b + 3] = ((double)r.w + 0.5) * (1.0 / 4294967296.0);
    }
    const float uc = (float)u[0] * tot;
    int c = kInitK - 1;
    float acc = 0.f;
    for (int q = 0; q < kInitK; ++q) {
        acc += w[q];
        if (uc < acc) { c = q; break; }
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int p = k / 2;
        const double rad = sqrt(-2.0 * log(u[2 + 2 * p]));
        const double th = 2.0 * kPi * u[3 + 2 * p];
        const float xi = (float)((k & 1) ? rad * sin(th) : rad * cos(th));
        const float rho = fminf(fmaxf(o[c * kInitComp + 8 + k], kRhoMin), kRhoMax);
        x.target[(long)i * D + k] = anc[k] + scl[k] * (o[c * kInitComp + 1 + k] + expf(rho) * xi);
    }
}

__global__ __launch_bounds__(256) void k_mix_sample(const InitExample *__restrict__ ex, int count,
                                                    const float *__restrict__ out, const float *__restrict__ anc,
                                                    const float *__restrict__ scl, int32_t *used)
{
    const int e = blockIdx.y;
    if (e >= count) return;
    const InitExample &x = ex[e];
    const float *o = out + (long)e * kInitOut;
    bool ok = true;
    for (int q = 0; q < kInitOut; ++q) ok &= __builtin_isfinite(o[q]);
    if (blockIdx.x == 0 && threadIdx.x == 0 && used) used[e] = ok ? 1 : 0;
    if (!ok) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= x.n) return;
    const float *a = anc + e * 8, *sc = scl + e * 8;
    switch (x.code) {
    case GROWTH1D: mix_sample_one<1>(x, i, o, a, sc); break;
    case RANGE2D: mix_sample_one<2>(x, i, o, a, sc); break;
    case CV4D: mix_sample_one<4>(x, i, o, a, sc); break;
    default: mix_sample_one<7>(x, i, o, a, sc); break;
    }
}

// Adam on the FP32 parameters, then the BF16 copies of the weight matrices
// (W3 padded to 128 rows; rows 120..127 stay zero).  c1 = 1 / (1 - b1^t) and
// c2 = 1 / (1 - b2^t) are the bias corrections of step t, computed by the
// host in FP64 (in FP32, 1 - b2^t cancels: relative error ~3e-5 at t = 2).
__global__ void k_adam(float *P, const float *__restrict__ G, float *mo, float *ve, long count, float lr, float b1,
                       float b2, float eps, float c1, float c2, uint16_t *w1b, uint16_t *w2b, uint16_t *w3b)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float g = G[i];
    const float m = b1 * mo[i] + (1.f - b1) * g;
    const float v = b2 * ve[i] + (1.f - b2) * g * g;
    mo[i] = m;
    ve[i] = v;
    const float mh = m * c1, vh = v * c2;
    const float p = P[i] - lr * mh / (sqrtf(vh) + eps);
    P[i] = p;
    if (i < kOffB1) w1b[i - kOffW1] = to_bf16(p);
    else if (i >= kOffW2 && i < kOffB2) w2b[i - kOffW2] = to_bf16(p);
    else if (i >= kOffW3 && i < kOffB3) w3b[i - kOffW3] = to_bf16(p);
}

// Example table of a batch plan's step t: sequence list[k] proposes its
// step-t particles from step t - 1.
__global__ void k_init_prep(const SeqDesc *__restrict__ seqs, const int *__restrict__ list, int count, int t,
                            InitExample *__restrict__ ex)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const SeqDesc &s = seqs[list[k]];
    InitExample x;
    x.m = s.m;
    const long nd = (long)s.n * s.d;
    x.xprev = s.parts + (long)(t - 2) * nd;
    x.phiprev = s.phis + (long)(t - 2) * s.n;
    x.z = s.z + (long)(t - 1) * s.m.obs_dim;
    x.mask = s.mask ? s.mask + (long)(t - 1) * s.m.n_obs : nullptr;
    x.target = s.parts + (long)(t - 1) * nd;
    x.np = s.n;
    x.n = s.use_proposal ? s.n : 0;  // nothing to draw for the others
    x.t = t;
    x.code = s.code;
    x.seq = 0;
    x.seed = s.seed;
    ex[k] = x;
}

// After sampling: the step's items take the sampled particles (init_given)
// where a sequence uses the proposal and its outputs were finite.
__global__ void k_init_apply(StepArgs<float> *items, const InitExample *__restrict__ ex,
                             const int32_t *__restrict__ used, int count)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) items[k].init_given = ex[k].n > 0 ? used[k] : 0;
}

// He initialisation: W ~ N(0, 2 / fan_in) from Philox4x32-10 (key seed,
// counter (i, 0, 0x696e6974, 0)) and Box-Muller; biases zero.
__global__ void k_init_he(float *P, uint64_t seed)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kInitParams) return;
    float fan = 0.f;
    if (i < kOffB1) fan = (float)kInitFeat;
    else if (i >= kOffW2 && i < kOffB2) fan = (float)kInitHidden;
    else if (i >= kOffW3 && i < kOffB3) fan = (float)kInitHidden;
    if (fan == 0.f) {
        P[i] = 0.f;
        return;
    }
    const U4 r = philox4x32_10(U4{(uint32_t)i, 0u, 0x696e6974u, 0u}, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = ((double)r.x + 0.5) * (1.0 / 4294967296.0), u2 = ((double)r.y + 0.5) * (1.0 / 4294967296.0);
    P[i] = (float)(sqrt(-2.0 * log(u1)) * cos(2.0 * kPi * u2) * sqrt(2.0 / fan));
}

// BF16 copies of the weight matrices from the FP32 parameters
__global__ void k_init_weights_bf16(const float *__restrict__ P, uint16_t *w1b, uint16_t *w2b, uint16_t *w3b)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kOffB1) w1b[i - kOffW1] = to_bf16(P[i]);
    else if (i >= kOffW2 && i < kOffB2) w2b[i - kOffW2] = to_bf16(P[i]);
    else if (i >= kOffW3 && i < kOffB3) w3b[i - kOffW3] = to_bf16(P[i]);
}

__global__ void k_fill_f32(float *p, float v, long count)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// out[0] = mean of v[0..n)
__global__ void k_mean_f32(const float *__restrict__ v, int n, float *out)
{
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += kWave) s += v[i];
    s = wave_sum(s);
    if (threadIdx.x == 0) out[0] = s / (float)n;
}

} // namespace smsq
