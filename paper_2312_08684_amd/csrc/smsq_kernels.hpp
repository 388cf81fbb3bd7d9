// Stein-MAP-Seq step kernels for gfx950.
//
// One workgroup owns one sequence and keeps its whole particle state in LDS
// for a time step: the previous particles' transition means, the current
// particles and their scores.  The file also holds the chip-wide
// particle-mode forward recursion, the lattice-mode recursion and the
// backtrack.  Every SVGD iteration (eq. SVGD_newupdate) is
//   (1) exact lower median of the pairwise squared distances (bandwidth
//       h = s med / ln N): all pairs, or those in a window around the
//       previous iteration's median, gathered in LDS and selected by a
//       ballot bisection on their bit patterns; radix selection over all
//       pairs when the window misses or overflows,
//   (2) per-particle score: observation gradient plus the log-sum-exp
//       transition-mixture gradient, with an online (running-max) softmax
//       over the previous particles,
//   (3) Stein direction phi_i = (1/N) sum_k [kappa_ik s_k + w_ik (x_i - x_k)]
//       with the RBF kernel kappa = exp(-D/h), w = (2/h) kappa, or the IMQ
//       and Matern-3/2 kernels of the kernel ablation (stein_kernel), then
//       x_i += eps phi_i for all i at once,
// and after the iterations the forward-recursion row of every particle
// (eq. forward_recursion) is a max-plus reduction over the previous step.
#pragma once

#include "smsq_models.hpp"

namespace smsq {

constexpr int kBins = 2048;          // radix-select histogram (11-bit digits)
constexpr int kMaxRowsPerThread = 2; // particles owned by one thread in the Stein pass

// IMQ (kernel 1) and Matern-3/2 (kernel 2) kernels of the kernel ablation
// (Sec. V-E) at squared distance dd: kap = f(dd), and w with
// grad_{x_k} kappa(x_i, x_k) = w (x_i - x_k), i.e. w = -2 f'(dd):
//   IMQ     f = (1 + dd/h)^(-1/2),                w = f^3 / h
//   Matern  f = (1 + a) e^(-a), a = sqrt(3 dd/h),  w = 3 e^(-a) / h
template <typename T>
__device__ __forceinline__ void stein_kernel(int kernel, T dd, T inv_h, T &kap, T &w)
{
    using R = RealOps<T>;
    if (kernel == 1) {
        const T v = (T)1 / R::sqrt_((T)1 + dd * inv_h);
        kap = v;
        w = v * v * v * inv_h;
    } else {
        const T av = R::sqrt_((T)3 * dd * inv_h);
        const T e = R::exp_(-av);
        kap = ((T)1 + av) * e;
        w = (T)3 * e * inv_h;
    }
}
constexpr int kMaxObs = 32;

// Device status bits: non-finite values; a multi-workgroup step whose
// workgroups did not all reach a barrier within the wait bound.
enum : uint32_t { STATUS_NONFINITE = 4u, STATUS_STALLED = 8u };

template <typename T> struct StepArgs {
    DevModel<T> m;
    // previous particles [batch][n_prev][d] (sequence stride x_prev_stride)
    const T *x_prev; long x_prev_stride;
    const T *log_w; long log_w_stride;      // may be null (uniform)
    const T *phi_prev; long phi_prev_stride; // may be null (zeros)
    const T *z; long z_stride;
    const uint8_t *mask; long mask_stride;  // may be null
    T *x; long x_stride;                    // [batch][n][d] in/out
    T *phi; long phi_stride;                // forward recursion outputs (may be null: no Viterbi)
    int32_t *psi; long psi_stride;
    uint8_t *flags; long flags_stride;      // may be null
    T *h_out; long h_stride;                // may be null
    uint32_t *status;
    int n_prev, n, t, n_iter, bw_mode, trans_mode, init_given, do_svgd, do_viterbi;
    int kernel;  // Stein kernel: 0 RBF, 1 IMQ, 2 Matern-3/2 (the matrix-core kernel takes 0 only)
    T step, bw_scale, tie_tol;
    uint64_t seed; uint32_t seq_offset;
};

__host__ __device__ constexpr long align16(long b) { return (b + 15) & ~15L; }

// LDS byte layout of a step workgroup.
template <typename T> struct StepLds {
    long off_x, off_s, off_m, off_c, off_hist, off_z, off_mask, off_red, total;
    __host__ __device__ StepLds(int n, int n_prev, int dp)
    {
        long o = 0;
        off_x = o; o += align16((long)n * dp * sizeof(T));
        off_s = o; o += align16((long)n * dp * sizeof(T));
        off_m = o; o += align16((long)n_prev * dp * sizeof(T));
        off_c = o; o += align16((long)n_prev * sizeof(T));
        off_hist = o; o += (long)kBins * sizeof(uint32_t);
        off_z = o; o += align16((long)kMaxObs * sizeof(T));
        off_mask = o; o += 64;
        off_red = o; o += 256;
        total = o;
    }
};

template <typename T, int DP> struct Vec { T v[DP]; };

template <typename T, int DP>
__device__ __forceinline__ void lds_load(const T *p, T (&r)[DP])
{
#pragma unroll
    for (int a = 0; a < DP; ++a) r[a] = p[a];
}

// ---------------------------------------------------------------------------
// (1) exact lower median of {|x_i - x_k|^2 : i < k} by radix selection.
// Pairs are visited as 64x64 tiles of the upper triangle; lane l of a wave
// takes row i = 64 ib + l and walks the tile's columns.
// ---------------------------------------------------------------------------
template <typename T, int D, int DP>
__device__ T block_median_sqdist(const T *sx, int n, uint32_t *hist, uint32_t *red)
{
    using KO = KeyOf<T>;
    using K = typename KO::K;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & (kWave - 1), wave = wave_id(), nwaves = nt / kWave;
    const uint32_t M = (uint32_t)((long)n * (n - 1) / 2);
    if (M == 0) return __builtin_nan("");
    uint32_t rank = (M - 1) / 2;
    K prefix = 0, pmask = 0;
    const int nb = (n + kWave - 1) / kWave;
    const int ntiles = nb * (nb + 1) / 2;
    for (int pass = 0; pass < KO::kPasses; ++pass) {
        const int shift = KO::shift(pass);
        const K dmask = ((K)1 << KO::width(pass)) - 1;
        for (int b = tid; b < kBins; b += nt) hist[b] = 0;
        __syncthreads();
        for (int tile = wave; tile < ntiles; tile += nwaves) {
            int ib = 0, rem = tile;
            while (rem >= nb - ib) { rem -= nb - ib; ++ib; }
            const int kb = ib + rem;
            const int i = ib * kWave + lane;
            T xi[DP];
            if (i < n) lds_load<T, DP>(sx + (long)i * DP, xi);
            const int k0 = kb * kWave;
            const int k1 = min(k0 + kWave, n);
            for (int k = k0; k < k1; ++k) {
                if (i < k && i < n) {
                    T xk[DP];
                    lds_load<T, DP>(sx + (long)k * DP, xk);
                    T dd = 0;
#pragma unroll
                    for (int a = 0; a < D; ++a) { const T r = xi[a] - xk[a]; dd += r * r; }
                    const K key = KO::key(dd);
                    if ((key & pmask) == prefix) atomicAdd(&hist[(uint32_t)((key >> shift) & dmask)], 1u);
                }
            }
        }
        __syncthreads();
        if (wave == 0) {
            constexpr int per = kBins / kWave;
            uint32_t cnt = 0;
            for (int q = 0; q < per; ++q) cnt += hist[lane * per + q];
            const uint32_t incl = wave_incl_scan(cnt, lane);
            const uint32_t excl = incl - cnt;
            if (lane == 0) { red[0] = 0; red[1] = 0; }
            __builtin_amdgcn_wave_barrier();
            if (rank >= excl && rank < incl) {
                uint32_t r = rank - excl;
                for (int q = 0; q < per; ++q) {
                    const uint32_t h = hist[lane * per + q];
                    if (r < h) { red[0] = (uint32_t)(lane * per + q); red[1] = r; break; }
                    r -= h;
                }
            }
        }
        __syncthreads();
        const uint32_t digit = red[0];
        rank = red[1];
        prefix |= (K)digit << shift;
        pmask |= dmask << shift;
        __syncthreads();
    }
    return KO::val(prefix);
}

// (1b) the same order statistic by one pass over a window: the pairs below
// lo are counted, those in [lo, hi] are gathered into buf (wave-aggregated
// appends, at most cap of them); when the rank falls inside the window the
// median is the matching order statistic of the gathered values.  Returns
// false, with the window's counts, when the rank lies outside it or it
// overflowed; the caller then takes the radix selection.  ALL gathers every
// pair (i, k) at slot k (k - 1) / 2 + i, with no counting.

__device__ __forceinline__ uint32_t uniform_key(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ uint64_t uniform_key(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// The r-th smallest (0-based) of the first cnt keys of buf, by one wave:
// the keys go to registers, S per lane, and the answer is built bit by bit
// below the common prefix of the smallest and largest key; bit b is set
// when at most r keys lie below the prefix with that bit set (ballot counts).
template <typename T, int S>
__device__ typename KeyOf<T>::K select_rank_wave(const T *buf, uint32_t cnt, uint32_t r, int lane)
{
    using KO = KeyOf<T>;
    using K = typename KO::K;
    constexpr int kBits = 8 * (int)sizeof(K);
    K key[S];
    K kmin = ~(K)0, kmax = 0;
#pragma unroll
    for (int sl = 0; sl < S; ++sl) {
        const uint32_t q = (uint32_t)(lane + sl * kWave);
        key[sl] = ~(K)0;
        if (q < cnt) {
            key[sl] = KO::key(buf[q]);
            kmin = key[sl] < kmin ? key[sl] : kmin;
            kmax = key[sl] > kmax ? key[sl] : kmax;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const K a = __shfl_xor(kmin, off, kWave), b = __shfl_xor(kmax, off, kWave);
        kmin = a < kmin ? a : kmin;
        kmax = b > kmax ? b : kmax;
    }
    // every lane holds the same extremes: make them scalar so that the
    // search below runs on scalar registers with scalar loop control
    kmin = uniform_key(kmin);
    kmax = uniform_key(kmax);
    const K diff = kmin ^ kmax;
    const int top = diff ? kBits - 1 - (sizeof(K) == 8 ? __builtin_clzll((unsigned long long)diff)
                                                       : __builtin_clz((uint32_t)diff)) : -1;
    K prefix = top >= kBits - 1 ? (K)0 : (kmin & ~((((K)1) << (top + 1)) - 1));
    for (int b = top; b >= 0; --b) {
        const K t = prefix | ((K)1 << b);
        uint64_t m[S];
#pragma unroll
        for (int sl = 0; sl < S; ++sl) m[sl] = __builtin_amdgcn_ballot_w64(key[sl] < t);
        uint32_t c = 0;
#pragma unroll
        for (int sl = 0; sl < S; ++sl) c += (uint32_t)__builtin_popcountll(m[sl]);
        if (c <= r) prefix = t;
    }
    return prefix;
}

template <typename T, int D, int DP, bool ALL>
__device__ bool window_median_sqdist(const T *sx, int n, T lo, T hi, T *buf, uint32_t cap, uint32_t *red, T &med,
                                     uint32_t &cnt_lo, uint32_t &cnt_in)
{
    using KO = KeyOf<T>;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & (kWave - 1), wave = wave_id(), nwaves = nt / kWave;
    const uint32_t M = (uint32_t)((long)n * (n - 1) / 2);
    const uint32_t rank = (M - 1) / 2;
    if (!ALL) {
        if (tid == 0) { red[2] = 0; red[3] = 0; }
        __syncthreads();
    }
    uint32_t below = 0;
    const int nb = (n + kWave - 1) / kWave;
    const int ntiles = nb * (nb + 1) / 2;
    for (int tile = wave; tile < ntiles; tile += nwaves) {
        int ib = 0, rem = tile;
        while (rem >= nb - ib) { rem -= nb - ib; ++ib; }
        const int kb = ib + rem;
        const int i = ib * kWave + lane;
        T xi[DP];
        if (i < n) lds_load<T, DP>(sx + (long)i * DP, xi);
        const int k0 = kb * kWave;
        const int k1 = min(k0 + kWave, n);
        for (int k = k0; k < k1; ++k) {
            const bool valid = i < k && i < n;
            T dd = 0;
            if (valid) {
                T xk[DP];
                lds_load<T, DP>(sx + (long)k * DP, xk);
#pragma unroll
                for (int a = 0; a < D; ++a) { const T r = xi[a] - xk[a]; dd += r * r; }
            }
            if (ALL) {
                if (valid) buf[(uint32_t)k * (uint32_t)(k - 1) / 2 + (uint32_t)i] = dd;
                continue;
            }
            below += (valid && dd < lo) ? 1u : 0u;
            const bool in = valid && dd >= lo && dd <= hi;
            const uint64_t m = __builtin_amdgcn_ballot_w64(in);
            if (m) {
                const int leader = (int)__builtin_ctzll(m);
                uint32_t base = 0;
                if (lane == leader) base = atomicAdd(&red[2], (uint32_t)__builtin_popcountll(m));
                base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
                const uint32_t pos = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                               __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                if (in && pos < cap) buf[pos] = dd;
            }
        }
    }
    if (ALL) {
        cnt_lo = 0;
        cnt_in = M;
        __syncthreads();
    } else {
        below = wave_sum(below);
        if (lane == 0) atomicAdd(&red[3], below);
        __syncthreads();
        cnt_in = red[2];
        cnt_lo = red[3];
        __syncthreads();
        if (cnt_in > cap || rank < cnt_lo || rank >= cnt_lo + cnt_in) return false;
    }
    if (wave == 0) {
        const uint32_t r = rank - cnt_lo;
        const uint32_t used = (cnt_in + kWave - 1) / kWave;
        typename KO::K v;
        if (used <= 1) v = select_rank_wave<T, 1>(buf, cnt_in, r, lane);
        else if (used <= 2) v = select_rank_wave<T, 2>(buf, cnt_in, r, lane);
        else if (used <= 4) v = select_rank_wave<T, 4>(buf, cnt_in, r, lane);
        else if (used <= 8) v = select_rank_wave<T, 8>(buf, cnt_in, r, lane);
        else if (used <= 16) v = select_rank_wave<T, 16>(buf, cnt_in, r, lane);
        else v = select_rank_wave<T, kBins * (int)sizeof(uint32_t) / (int)sizeof(T) / kWave>(buf, cnt_in, r, lane);
        if (lane == 0) *(T *)(red + 4) = KO::val(v);
    }
    __syncthreads();
    med = *(const T *)(red + 4);
    __syncthreads();
    return true;
}

template <typename T> __device__ __forceinline__ T bandwidth_from_median(T med, int n, T bw_scale)
{
    T h = (n > 1) ? bw_scale * med / RealOps<T>::log_((T)n) : (T)0;
    if (!(h > (T)0) || !RealOps<T>::finite(h)) h = (T)1;
    return h;
}

// ---------------------------------------------------------------------------
// The fused step kernel: initial particles, SVGD iterations, forward recursion.
// ---------------------------------------------------------------------------
template <typename T, int KIND, int D>
__global__ __launch_bounds__(1024) void k_step(StepArgs<T> a)
{
    using F = Family<T, KIND, D>;
    using R = RealOps<T>;
    constexpr int DP = dpad(D);
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = a.n, np = a.n_prev;
    const StepLds<T> L(n, np, DP);
    T *sx = (T *)(smem + L.off_x);
    T *ss = (T *)(smem + L.off_s);
    T *sm = (T *)(smem + L.off_m);
    T *sc = (T *)(smem + L.off_c);
    uint32_t *hist = (uint32_t *)(smem + L.off_hist);
    T *sz = (T *)(smem + L.off_z);
    uint8_t *smask = smem + L.off_mask;
    uint32_t *red = (uint32_t *)(smem + L.off_red);
    T *redT = (T *)(smem + L.off_red + 64);

    const int b = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    const DevModel<T> &m = a.m;
    const T *xprev = a.x_prev + (long)b * a.x_prev_stride;
    T *xg = a.x + (long)b * a.x_stride;

    // observation of this step
    for (int o = tid; o < m.obs_dim; o += nt) sz[o] = a.z[(long)b * a.z_stride + o];
    const uint8_t *mk = nullptr;
    if (a.mask) {
        for (int o = tid; o < m.n_obs; o += nt) smask[o] = a.mask[(long)b * a.mask_stride + o];
        mk = smask;
    }
    // Particles and transition means are kept relative to a centre, the
    // transition mean of the first previous particle, so that the updates
    // and pairwise differences keep their precision when the cloud sits far
    // from the origin; the model densities see centre + offset.
    T cen[D];
    {
        T xp[D];
#pragma unroll
        for (int c = 0; c < D; ++c) xp[c] = xprev[c];
        F::mean(m, a.t, xp, cen);
    }
    // transition means of the previous particles, centred and scaled to log2
    // units, and their log-weights (log2 units)
    T rs[DP];
#pragma unroll
    for (int c = 0; c < DP; ++c) rs[c] = c < D ? m.rs[c] : (T)0;
    for (int j = tid; j < np; j += nt) {
        T xp[D], mu[D];
#pragma unroll
        for (int c = 0; c < D; ++c) xp[c] = xprev[(long)j * D + c];
        F::mean(m, a.t, xp, mu);
#pragma unroll
        for (int c = 0; c < DP; ++c) sm[(long)j * DP + c] = c < D ? (mu[c] - cen[c]) * rs[c] : (T)0;
        const T lw = a.log_w ? a.log_w[(long)b * a.log_w_stride + j] : -R::log_((T)np);
        sc[j] = lw * (T)kLog2e;
    }
    // initial particles
    for (int i = tid; i < n; i += nt) {
        T xi[D];
        if (a.init_given) {
#pragma unroll
            for (int c = 0; c < D; ++c) xi[c] = xg[(long)i * D + c] - cen[c];
        } else {
            T xp[D], mu[D];
            const int j = i % np;
#pragma unroll
            for (int c = 0; c < D; ++c) xp[c] = xprev[(long)j * D + c];
            F::mean(m, a.t, xp, mu);
            double nz[D];
            normals<D>(a.seed, a.seq_offset + (uint32_t)b, (uint32_t)a.t, (uint32_t)i, nz);
#pragma unroll
            for (int c = 0; c < D; ++c) xi[c] = (mu[c] - cen[c]) + m.sqrt_q[c] * (T)nz[c];
        }
#pragma unroll
        for (int c = 0; c < DP; ++c) sx[(long)i * DP + c] = c < D ? xi[c] : (T)0;
    }
    __syncthreads();

    // mean of the transition means (paper-literal score reading)
    T mbar_all[D];
#pragma unroll
    for (int c = 0; c < D; ++c) mbar_all[c] = 0;
    if (a.do_svgd && a.trans_mode == 1) {
        for (int c = 0; c < D; ++c) {
            T part = 0;
            for (int j = tid; j < np; j += nt) part += sm[(long)j * DP + c] / rs[c];
            part = wave_sum(part);
            if ((tid & (kWave - 1)) == 0) redT[tid / kWave] = part;
            __syncthreads();
            T tot = 0;
            for (int w = 0; w < nt / kWave; ++w) tot += redT[w];
            mbar_all[c] = tot / (T)np;
            __syncthreads();
        }
    }

    const T inv_n = (T)1 / (T)n;
    T h = (T)1;
    // median selection: all pairs gathered when they fit the window buffer,
    // else a window around the previous iteration's median whose relative
    // half-width adapts to keep the gathered count modest; radix selection
    // when the window misses or overflows
    const uint32_t n_pairs = (uint32_t)((long)n * (n - 1) / 2);
    const uint32_t cap = min((uint32_t)(kBins * sizeof(uint32_t) / sizeof(T)), (uint32_t)(4 * nt));
    T med_prev = (T)0, wrel = (T)0.02;
    bool have_prev = false;
    for (int it = 0; a.do_svgd && it < a.n_iter; ++it) {
        // (1) bandwidth
        if (a.bw_mode == 0 || it == 0) {
            T med = (T)0;
            uint32_t clo = 0, cin = 0;
            bool ok = false;
            if (n_pairs >= 1 && n_pairs <= cap) {
                ok = window_median_sqdist<T, D, DP, true>(sx, n, (T)0, R::inf(), (T *)hist, cap, red, med, clo, cin);
            } else if (n_pairs > cap && have_prev) {
                ok = window_median_sqdist<T, D, DP, false>(sx, n, med_prev * ((T)1 - wrel), med_prev * ((T)1 + wrel),
                                                    (T *)hist, cap, red, med, clo, cin);
                const uint32_t rank = (n_pairs - 1) / 2;
                if (ok) wrel = cin < cap / 8 ? wrel * (T)1.5 : (cin > cap / 2 ? wrel * (T)0.7 : wrel);
                else if (cin > cap) wrel *= (T)0.5;
                else if (rank < clo || rank >= clo + cin) wrel *= (T)2;
                if (wrel > (T)0.5) wrel = (T)0.5;
            }
            if (!ok) med = block_median_sqdist<T, D, DP>(sx, n, hist, red);
            med_prev = med;
            have_prev = med > (T)0 && R::finite(med);
            h = bandwidth_from_median(med, n, a.bw_scale);
        }
        if (a.h_out && tid == 0) a.h_out[(long)b * a.h_stride + it] = h;

        // (2) scores
        for (int k = tid; k < n; k += nt) {
            T xk[DP], xa[D];
            lds_load<T, DP>(sx + (long)k * DP, xk);
#pragma unroll
            for (int c = 0; c < D; ++c) xa[c] = xk[c] + cen[c];
            T g[D];
            F::grad(m, sz, mk, xa, g);
            T mb[D];
            if (a.trans_mode == 0) {
                T xs[DP];
#pragma unroll
                for (int c = 0; c < DP; ++c) xs[c] = xk[c] * rs[c];
                T mx = -R::inf(), sum = 0, acc[D];
#pragma unroll
                for (int c = 0; c < D; ++c) acc[c] = 0;
                constexpr int CH = DP >= 8 ? 4 : 8;
                int j0 = 0;
                for (; j0 + CH <= np; j0 += CH) {
                    T av[CH];
#pragma unroll
                    for (int u = 0; u < CH; ++u) {
                        T mj[DP];
                        lds_load<T, DP>(sm + (long)(j0 + u) * DP, mj);
                        T q2 = 0;
#pragma unroll
                        for (int c = 0; c < D; ++c) { const T r = xs[c] - mj[c]; q2 += r * r; }
                        av[u] = sc[j0 + u] - q2;
                    }
                    T cm = av[0];
#pragma unroll
                    for (int u = 1; u < CH; ++u) cm = av[u] > cm ? av[u] : cm;
                    const T nm = cm > mx ? cm : mx;
                    const T sf = R::exp2_(mx - nm);
                    sum *= sf;
#pragma unroll
                    for (int c = 0; c < D; ++c) acc[c] *= sf;
                    mx = nm;
#pragma unroll
                    for (int u = 0; u < CH; ++u) {
                        const T e = R::exp2_(av[u] - mx);
                        sum += e;
                        T mj[DP];
                        lds_load<T, DP>(sm + (long)(j0 + u) * DP, mj);
#pragma unroll
                        for (int c = 0; c < D; ++c) acc[c] += e * mj[c];
                    }
                }
                for (; j0 < np; ++j0) {
                    T mj[DP];
                    lds_load<T, DP>(sm + (long)j0 * DP, mj);
                    T q2 = 0;
#pragma unroll
                    for (int c = 0; c < D; ++c) { const T r = xs[c] - mj[c]; q2 += r * r; }
                    const T av = sc[j0] - q2;
                    const T nm = av > mx ? av : mx;
                    const T sf = R::exp2_(mx - nm);
                    const T e = R::exp2_(av - nm);
                    sum = sum * sf + e;
#pragma unroll
                    for (int c = 0; c < D; ++c) acc[c] = acc[c] * sf + e * mj[c];
                    mx = nm;
                }
                const T isum = (T)1 / sum;
#pragma unroll
                for (int c = 0; c < D; ++c) mb[c] = acc[c] * isum / rs[c];
            } else {
#pragma unroll
                for (int c = 0; c < D; ++c) mb[c] = mbar_all[c];
            }
#pragma unroll
            for (int c = 0; c < DP; ++c)
                ss[(long)k * DP + c] = c < D ? g[c] - (xk[c] - mb[c]) * m.inv_q[c] : (T)0;
        }
        __syncthreads();

        // (3) Stein direction and synchronous update
        const T beta = (T)kLog2e / h;
        const T c2 = (T)2 / h;
        const T inv_h = (T)1 / h;
        T phi[kMaxRowsPerThread][D];
#pragma unroll
        for (int r = 0; r < kMaxRowsPerThread; ++r) {
            const int i = tid + r * nt;
            if (i >= n) break;
            T xi[DP];
            lds_load<T, DP>(sx + (long)i * DP, xi);
            T as[D], ar[D];
#pragma unroll
            for (int c = 0; c < D; ++c) { as[c] = 0; ar[c] = 0; }
            for (int k = 0; k < n; ++k) {
                T xk[DP], sk[DP];
                lds_load<T, DP>(sx + (long)k * DP, xk);
                lds_load<T, DP>(ss + (long)k * DP, sk);
                T df[D], dd = 0;
#pragma unroll
                for (int c = 0; c < D; ++c) { df[c] = xi[c] - xk[c]; dd += df[c] * df[c]; }
                T kap, w;
                if (a.kernel == 0) {
                    kap = R::exp2_(-beta * dd);
                    w = kap;  // times 2/h below
                } else {
                    stein_kernel<T>(a.kernel, dd, inv_h, kap, w);
                }
#pragma unroll
                for (int c = 0; c < D; ++c) { as[c] += kap * sk[c]; ar[c] += w * df[c]; }
            }
            const T cw = a.kernel == 0 ? c2 : (T)1;
#pragma unroll
            for (int c = 0; c < D; ++c) phi[r][c] = (as[c] + cw * ar[c]) * inv_n;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kMaxRowsPerThread; ++r) {
            const int i = tid + r * nt;
            if (i >= n) break;
#pragma unroll
            for (int c = 0; c < D; ++c) sx[(long)i * DP + c] += a.step * phi[r][c];
        }
        __syncthreads();
    }

    // write particles back; flag non-finite values
    bool bad = false;
    for (int i = tid; a.do_svgd && i < n; i += nt) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const T v = sx[(long)i * DP + c] + cen[c];
            bad |= !R::finite(v);
            xg[(long)i * D + c] = v;
        }
    }

    if (a.do_viterbi) {
        // forward recursion: c_ij = A_ij + phi_prev(j), A_ij = log_z - ln2 * |xs_i - ms_j|^2
        for (int j = tid; j < np; j += nt)
            sc[j] = a.phi_prev ? a.phi_prev[(long)b * a.phi_prev_stride + j] : (T)0;
        __syncthreads();
        for (int i = tid; i < n; i += nt) {
            T xi[DP], xs[DP];
            lds_load<T, DP>(sx + (long)i * DP, xi);
#pragma unroll
            for (int c = 0; c < DP; ++c) xs[c] = xi[c] * rs[c];
            ArgBest<T> ab{-R::inf(), -R::inf(), 0};
            bool nan_seen = false;
            for (int j = 0; j < np; ++j) {
                T mj[DP];
                lds_load<T, DP>(sm + (long)j * DP, mj);
                T q2 = 0;
#pragma unroll
                for (int c = 0; c < D; ++c) { const T r = xs[c] - mj[c]; q2 += r * r; }
                const T A = m.log_z - (T)kLn2 * q2;
                const T cij = A + sc[j];
                nan_seen |= (cij != cij);
                if (j == 0) { ab.best = cij; ab.arg = 0; }
                else argbest_push(ab, cij, j);
            }
            T xa[D];
#pragma unroll
            for (int c = 0; c < D; ++c) xa[c] = xi[c] + cen[c];
            const T ell = F::loglik(m, sz, mk, xa);
            const T ph = ab.best + ell;
            nan_seen |= (ph != ph);
            bad |= nan_seen;
            a.phi[(long)b * a.phi_stride + i] = ph;
            a.psi[(long)b * a.psi_stride + i] = ab.arg;
            if (a.flags) {
                const T sc_ = ab.best > (T)1 || ab.best < (T)-1 ? (ab.best < 0 ? -ab.best : ab.best) : (T)1;
                a.flags[(long)b * a.flags_stride + i] = (np > 1 && ab.second >= ab.best - a.tie_tol * sc_) ? 1 : 0;
            }
        }
    }
    if (bad) atomicOr(a.status, STATUS_NONFINITE);
}

// ---------------------------------------------------------------------------
// Lattice-mode forward recursion: two waves per row i (halves of j,
// coalesced), merged through LDS.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_viterbi_lattice(int n, int n_prev, const T *__restrict__ A,
                                                         const T *__restrict__ ell,
                                                         const T *__restrict__ phi_prev, T *phi,
                                                         int32_t *psi, uint8_t *flags, T tie_tol,
                                                         uint32_t *status)
{
    using R = RealOps<T>;
    constexpr int kSplit = 2;                  // waves per row
    constexpr int kRowsPerBlock = 4 / kSplit;  // four waves per workgroup
    __shared__ T sbest[4], ssecond[4];
    __shared__ int sarg[4];
    // lattice blockIdx.y of a batch: consecutive [n][n_prev] lattices, [n]
    // observation terms, [n_prev] previous scores and [n] outputs
    {
        const long bb = blockIdx.y;
        A += bb * (long)n * n_prev;
        ell += bb * n;
        phi_prev += bb * n_prev;
        phi += bb * n;
        psi += bb * n;
        if (flags) flags += bb * n;
    }
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int part = w % kSplit;
    const int i = blockIdx.x * kRowsPerBlock + w / kSplit;
    const bool live = i < n;
    ArgBest<T> ab{-R::inf(), -R::inf(), 0x7fffffff};
    bool nan_seen = false;
    // 16-byte loads, four per lane in flight (4 KB per wave), when the rows
    // allow; each wave takes one contiguous part of the row and each lane
    // visits its indices in ascending order, so the first maximum wins within
    // a lane and the merges keep the lowest index
    constexpr int V = 16 / (int)sizeof(T);
    typedef T vec_t __attribute__((ext_vector_type(V)));
    const bool vec = n_prev % V == 0 && ((uintptr_t)A % 16) == 0 && ((uintptr_t)phi_prev % 16) == 0;
    if (live && vec) {
        const int nv = n_prev / V;
        const int lo = (int)((long)nv * part / kSplit), hi = (int)((long)nv * (part + 1) / kSplit);
        const vec_t *rv = (const vec_t *)(A + (long)i * n_prev);
        const vec_t *pv = (const vec_t *)phi_prev;
        bool first = true;
        for (int v0 = lo + lane; v0 < hi; v0 += 4 * kWave) {
            vec_t a4[4], p4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int v = v0 + u * kWave;
                if (v < hi) {
                    a4[u] = __builtin_nontemporal_load(rv + v);
                    p4[u] = pv[v];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int v = v0 + u * kWave;
                if (v < hi) {
#pragma unroll
                    for (int e = 0; e < V; ++e) {
                        const T c = a4[u][e] + p4[u][e];
                        const int j = v * V + e;
                        nan_seen |= (c != c);
                        if (first) { ab.best = c; ab.arg = j; first = false; }
                        else argbest_push(ab, c, j);
                    }
                }
            }
        }
    } else if (live) {
        const int lo = (int)((long)n_prev * part / kSplit), hi = (int)((long)n_prev * (part + 1) / kSplit);
        const T *row = A + (long)i * n_prev;
        bool first = true;
        for (int j = lo + lane; j < hi; j += kWave) {
            const T c = row[j] + phi_prev[j];
            nan_seen |= (c != c);
            if (first) { ab.best = c; ab.arg = j; first = false; }
            else argbest_push(ab, c, j);
        }
    }
    ab = wave_argbest(ab);
    if (lane == 0) { sbest[w] = ab.best; ssecond[w] = ab.second; sarg[w] = ab.arg; }
    __syncthreads();
    if (live && part == 0 && lane == 0) {
        for (int h = 1; h < kSplit; ++h) ab = argbest_merge(ab, ArgBest<T>{sbest[w + h], ssecond[w + h], sarg[w + h]});
        const T e = ell[i];
        const T ph = ab.best + e;
        phi[i] = ph;
        psi[i] = ab.arg;
        if (flags) {
            const T mag = ab.best < 0 ? -ab.best : ab.best;
            const T sc = mag > (T)1 ? mag : (T)1;
            flags[i] = (n_prev > 1 && ab.second >= ab.best - tie_tol * sc) ? 1 : 0;
        }
        nan_seen |= (e != e) || (ph != ph);
    }
    if (__any(nan_seen) && lane == 0) atomicOr(status, STATUS_NONFINITE);
}

// ---------------------------------------------------------------------------
// Particle-mode forward recursion over the whole chip: c_ij = log N(x_t^i;
// f_t(x_{t-1}^j), diag q) + phi_{t-1}(j), psi_i = lowest argmax_j c_ij,
// phi_i = log p(z_t | x_t^i) + c_{i psi_i} (eq. forward_recursion).  Each
// workgroup evaluates the transition means of all previous particles once
// into LDS (centred on f_t(x_{t-1}^0) and scaled by sqrt(log2 e / (2 q)), as
// in the step kernels); then each row i is taken by two waves, one per half
// of the previous particles (merged through LDS, the lower half winning
// equal scores).  A lane walks its indices j in ascending order in kChains
// independent chains (j = lane + 64 (kChains u + v)), so that the loads and
// arithmetic of different chains overlap; chains and lanes merge with the
// lowest index winning equal scores, and the first lane adds the observation
// term.  FLAGS: the runner-up is tracked for the tie flags.  Bound by the
// vector ALU: (2d + 4) flops and one compare per edge; the LDS table is
// read, never HBM, inside the edge loop.  NT threads per workgroup: 1024
// for small states, so that one table serves eight rows at a time.
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ void argbest_push_best(ArgBest<T> &a, T c, int j)
{
    const bool up = c > a.best;
    a.best = up ? c : a.best;
    a.arg = up ? j : a.arg;
}

template <typename T, int KIND, int D, int NT, bool FLAGS>
__global__ __launch_bounds__(NT) void k_viterbi_particle_wide(DevModel<T> m, int t, int n, int n_prev,
                                                               const T *__restrict__ x_prev,
                                                               const T *__restrict__ phi_prev,
                                                               const T *__restrict__ z, const uint8_t *mask,
                                                               const T *__restrict__ x, T *phi, int32_t *psi,
                                                               uint8_t *flags, T tie_tol, uint32_t *status)
{
    using F = Family<T, KIND, D>;
    using R = RealOps<T>;
    constexpr int DP = dpad(D);
    constexpr int kChains = 4;
    constexpr int kPairs = NT / kWave / 2;   // rows at a time per workgroup
    extern __shared__ __align__(16) unsigned char smem[];
    T *sm = (T *)smem;                                       // [n_prev][DP] scaled centred means
    T *sp = (T *)(smem + align16((long)n_prev * DP * sizeof(T)));   // [n_prev] phi_{t-1}
    __shared__ T s_best[NT / kWave], s_second[NT / kWave];
    __shared__ int s_arg[NT / kWave];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & (kWave - 1), w = wave_id(), half = w & 1;

    T cen[D], rs[D];
    {
        T xp[D];
#pragma unroll
        for (int c = 0; c < D; ++c) xp[c] = x_prev[c];
        F::mean(m, t, xp, cen);
    }
#pragma unroll
    for (int c = 0; c < D; ++c) rs[c] = m.rs[c];
    for (int j = tid; j < n_prev; j += nt) {
        T xp[D], mu[D];
#pragma unroll
        for (int c = 0; c < D; ++c) xp[c] = x_prev[(long)j * D + c];
        F::mean(m, t, xp, mu);
#pragma unroll
        for (int c = 0; c < DP; ++c) sm[(long)j * DP + c] = c < D ? (mu[c] - cen[c]) * rs[c] : (T)0;
        sp[j] = phi_prev[j];
    }
    __syncthreads();

    bool nan_seen = false;
    const int jmid = (n_prev + 1) / 2;
    const int j0 = half ? jmid : 0, j1 = half ? n_prev : jmid;
    // the same trip count in every wave of the workgroup (barriers inside)
    for (int ib = blockIdx.x * kPairs; ib < n; ib += gridDim.x * kPairs) {
        const int i = ib + (w >> 1);
        const bool live = i < n;
        ArgBest<T> a{-R::inf(), -R::inf(), 0x7fffffff};
        T xi[D];
        if (live) {
            T xs[D];
#pragma unroll
            for (int c = 0; c < D; ++c) {
                xi[c] = x[(long)i * D + c];
                xs[c] = (xi[c] - cen[c]) * rs[c];
            }
            ArgBest<T> ab[kChains];
#pragma unroll
            for (int v = 0; v < kChains; ++v) ab[v] = ArgBest<T>{-R::inf(), -R::inf(), 0x7fffffff};
            for (int jb = j0 + lane; jb < j1; jb += kWave * kChains) {
#pragma unroll
                for (int v = 0; v < kChains; ++v) {
                    const int j = jb + kWave * v;
                    if (j < j1) {
                        T mj[DP];
                        lds_load<T, DP>(sm + (long)j * DP, mj);
                        T q2 = 0;
#pragma unroll
                        for (int c = 0; c < D; ++c) { const T r = xs[c] - mj[c]; q2 += r * r; }
                        const T cij = (m.log_z - (T)kLn2 * q2) + sp[j];
                        nan_seen |= (cij != cij);
                        if (FLAGS) argbest_push(ab[v], cij, j);
                        else argbest_push_best(ab[v], cij, j);
                    }
                }
            }
            a = ab[0];
#pragma unroll
            for (int v = 1; v < kChains; ++v) a = argbest_merge(a, ab[v]);
            a = wave_argbest(a);
            if (lane == 0) {
                s_best[w] = a.best;
                s_second[w] = a.second;
                s_arg[w] = a.arg;
            }
        }
        __syncthreads();
        if (live && half == 0 && lane == 0) {
            a = argbest_merge(a, ArgBest<T>{s_best[w + 1], s_second[w + 1], s_arg[w + 1]});
            const T ell = F::loglik(m, z, mask, xi);
            const T ph = a.best + ell;
            phi[i] = ph;
            psi[i] = a.arg == 0x7fffffff ? 0 : a.arg;
            if (flags) {
                const T mag = a.best < 0 ? -a.best : a.best;
                const T sc = mag > (T)1 ? mag : (T)1;
                flags[i] = (n_prev > 1 && a.second >= a.best - tie_tol * sc) ? 1 : 0;
            }
            nan_seen |= (ell != ell) || (ph != ph);
        }
        __syncthreads();
    }
    if (__any(nan_seen) && lane == 0) atomicOr(status, STATUS_NONFINITE);
}

// ---------------------------------------------------------------------------
// Particle-mode forward recursion, rows in blocks of RP.  The
// edge score above is ranked in log2 units, in one fixed direct form: c'_ij =
// s_j - |y_i - m_j|^2 with s_j = (log_z + phi_{t-1}(j)) log2 e, the particles
// y_i and transition means m_j centred on f_t(x_{t-1}^0) and scaled by
// sqrt(log2 e / (2 q)), so that c'_ij = c_ij log2 e; each squared coordinate
// difference is one fused multiply-subtract, 2d instructions per edge.  The
// winner's score is taken back to natural-log units (c = ln2 c').  LDS holds
// the workgroup's table tile by tile: for each run of kTile consecutive
// indices, D + 1 arrays of kTile entries (the means coordinate by coordinate,
// then s_j), so that one base address with constant offsets serves a whole
// tile; npad is n_prev rounded up to a multiple of rows_table_align(RP).  Tiles
// that start at or beyond n_prev are skipped, and the last one is padded to its
// end with m = 0 and score -inf, which never wins, so no edge needs a bounds
// check.  A workgroup takes RP = 4, 8 or 16 rows at a time (the launch picks
// the largest that still gives every compute unit a workgroup): lane l of wave
// w takes row l % RP and, of the previous particles, the w-th sixteenth of the
// table in tiles of 8 * 64 / RP indices, eight consecutive ones per lane group
// l / RP.  Per tile a lane takes the maximum of its eight scores and keeps the
// first tile that raised its running maximum; that tile's scores are evaluated
// again at the end (the same arithmetic, hence the same values) to find the
// lowest index reaching it.  Lanes of a row merge by shuffles, the 16 waves
// through LDS (read by all of wave 0, then shuffles again), equal scores always
// going to the lower index.  A non-finite scaled coordinate or a NaN / +inf
// score offset (checked once per table entry and per row) is the only way to a
// NaN score; then the workgroup walks its edges one by one, skipping the
// padding and flagging NaN scores, as the kernel above does.  FLAGS: each
// lane also keeps the best of its other tiles' maxima and, at the end, of
// the winning tile's other scores (its runner-up over all its indices but
// the winner); merges keep the better of the winner's runner-up and the
// loser's best; the tie test runs in log2 units.  Bound by the
// vector ALU: 2d instructions per edge, and 9 per lane and tile of eight for
// its maximum, the compare, the two selects and the tile index and address.
// ---------------------------------------------------------------------------
constexpr int kRowsWaves = 16;       // waves per workgroup
constexpr int kRowsPer = 8;          // consecutive edges per lane and tile
__host__ __device__ constexpr int rows_tile(int rp) { return kRowsPer * (kWave / rp); }
__host__ __device__ constexpr int rows_table_align(int rp) { return kRowsWaves * rows_tile(rp); }

template <typename T> __device__ __forceinline__ T fma_(T a, T b, T c);
template <> __device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename T> __device__ __forceinline__ T vmax_(T a, T b);
template <> __device__ __forceinline__ float vmax_(float a, float b) { return __builtin_fmaxf(a, b); }
template <> __device__ __forceinline__ double vmax_(double a, double b) { return __builtin_fmax(a, b); }

typedef float lds_f4 __attribute__((ext_vector_type(4)));
typedef double lds_d2 __attribute__((ext_vector_type(2)));

// K consecutive table entries from a 16-byte aligned LDS address
template <int K> __device__ __forceinline__ void lds_run(const float *p, float (&v)[K])
{
#pragma unroll
    for (int k = 0; k < K; k += 4) {
        const lds_f4 q = *(const lds_f4 *)(p + k);
        v[k] = q[0]; v[k + 1] = q[1]; v[k + 2] = q[2]; v[k + 3] = q[3];
    }
}
template <int K> __device__ __forceinline__ void lds_run(const double *p, double (&v)[K])
{
#pragma unroll
    for (int k = 0; k < K; k += 2) {
        const lds_d2 q = *(const lds_d2 *)(p + k);
        v[k] = q[0]; v[k + 1] = q[1];
    }
}

// keeps (v, j) or takes (vo, jo): the larger score, the lower index among
// equal ones; NaN never taken (branch-free)
template <typename T> __device__ __forceinline__ void take_better(T &v, int &j, T vo, int jo)
{
    const bool b = (vo > v) | ((vo == v) & (jo < j));
    v = b ? vo : v;
    j = b ? jo : j;
}

// the same with runner-ups (the best score over the other indices): the
// winner keeps the better of its runner-up and the loser's best
template <typename T> __device__ __forceinline__ void take_better(T &v, int &j, T &r, T vo, int jo, T ro)
{
    const bool b = (vo > v) | ((vo == v) & (jo < j));
    const T lose = b ? v : vo;
    const T keep = b ? ro : r;
    v = b ? vo : v;
    j = b ? jo : j;
    r = vmax_(keep, lose);
}

// log2-unit scores of K edges of row y: p points at the first of them in
// the coordinate-0 array of a tile of TILE indices
template <typename T, int D, int K, int TILE>
__device__ __forceinline__ void row_edge_scores(const T *p, const T (&y)[D], T (&c)[K])
{
    lds_run<K>(p + D * TILE, c);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        T mv[K];
        lds_run<K>(p + a * TILE, mv);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const T r = y[a] - mv[k];
            c[k] = fma_(-r, r, c[k]);
        }
    }
}

template <typename T, int KIND, int D, int RP, bool FLAGS>
__global__ __launch_bounds__(kRowsWaves * kWave) void k_viterbi_particle_rows(
    DevModel<T> m, int t, int n, int n_prev, int npad, const T *__restrict__ x_prev, const T *__restrict__ phi_prev,
    const T *__restrict__ z, const uint8_t *mask, const T *__restrict__ x, T *phi, int32_t *psi, uint8_t *flags,
    T tie_tol, uint32_t *status)
{
    using F = Family<T, KIND, D>;
    using R = RealOps<T>;
    constexpr int NT = kRowsWaves * kWave;
    constexpr int kChunk = 4;                         // table entries per thread in flight
    constexpr int kTile = rows_tile(RP);
    extern __shared__ __align__(16) unsigned char smem[];
    T *tab = (T *)smem;                               // [npad / kTile][D + 1][kTile]
    __shared__ T s_v[kRowsWaves][RP];
    __shared__ int s_j[kRowsWaves][RP];
    __shared__ T s_r[FLAGS ? kRowsWaves : 1][RP];       // runner-ups (tie flags)
    __shared__ T s_z[kMaxObs];
    __shared__ uint8_t s_mask[kMaxObs];
    __shared__ int s_bad[kRowsWaves];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = wave_id();
    const int rl = lane & (RP - 1), grp = lane / RP;
    const int nrb = (n + RP - 1) / RP;

    // this workgroup's first rows and the centre, loaded before the table
    T xn[D];
    {
        const int i = blockIdx.x * RP + rl;
#pragma unroll
        for (int a = 0; a < D; ++a) xn[a] = i < n ? x[(long)i * D + a] : (T)0;
    }
    T xp0[D], cen[D], rs[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        xp0[a] = x_prev[a];
        rs[a] = m.rs[a];
    }
    // the observation, staged in LDS after the table loads are in flight
    const T zr = tid < m.obs_dim ? z[tid] : (T)0;
    const uint8_t mr = mask && tid < m.n_obs ? mask[tid] : (uint8_t)0;
    const int span = npad / kRowsWaves;               // this wave's share, a multiple of kTile
    const int nfill = (n_prev + kTile - 1) / kTile * kTile;   // entries the tiles read
    bool bad = false;
    for (int j0 = 0; j0 < nfill; j0 += kChunk * NT) {
        T xv[kChunk][D], pv[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            // clamped, so that every load is unconditional; padding is chosen
            // below (32-bit offsets: n_prev is bounded by the LDS)
            const int j = min(j0 + u * NT + tid, n_prev - 1);
#pragma unroll
            for (int a = 0; a < D; ++a) xv[u][a] = x_prev[j * D + a];
            pv[u] = phi_prev[j];
        }
        if (j0 == 0) F::mean(m, t, xp0, cen);
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            // every entry computed (from a clamped, valid index), padding
            // selected, only the store guarded: no divergent branches; the
            // chunk's tail past the table is cut workgroup-uniformly
            if (j0 + u * NT >= nfill) break;
            const int j = j0 + u * NT + tid;
            const bool real = j < n_prev;
            T mu[D];
            F::mean(m, t, xv[u], mu);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const T v = (mu[a] - cen[a]) * rs[a];
                bad |= real & !R::finite(v);
                mu[a] = real ? v : (T)0;
            }
            const T sv = (m.log_z + pv[u]) * (T)kLog2e;
            bad |= real & ((sv != sv) | (sv == R::inf()));
            const T s = real ? sv : -R::inf();
            if (j < nfill) {
                T *e = tab + (j / kTile) * (D + 1) * kTile + (j % kTile);
#pragma unroll
                for (int a = 0; a < D; ++a) e[a * kTile] = mu[a];
                e[D * kTile] = s;
            }
        }
    }
    if (tid < m.obs_dim) s_z[tid] = zr;
    if (tid < m.n_obs) s_mask[tid] = mr;
    {
        const bool wbad = __any(bad);
        if (lane == 0) s_bad[w] = wbad;
        __syncthreads();
        bad = false;
#pragma unroll
        for (int h = 0; h < kRowsWaves; ++h) bad |= s_bad[h] != 0;
    }

    const int jw0 = w * span;                         // this wave's first index
    const int jw = jw0 + grp * kRowsPer;              // this lane's first index
    // this lane's entries of the wave's first tile
    const T *tw = tab + (long)(jw0 / kTile) * (D + 1) * kTile + grp * kRowsPer;
    const uint8_t *mk = mask ? s_mask : nullptr;
    bool nan_seen = false;
    for (int rb = blockIdx.x; rb < nrb; rb += gridDim.x) {
        const int i = rb * RP + rl;
        const bool live = i < n;
        T xi[D], y[D];
        bool rbad = false;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            xi[a] = xn[a];
            y[a] = live ? (xi[a] - cen[a]) * rs[a] : (T)0;
            rbad |= !R::finite(y[a]);
        }
        {   // the next pass's rows, in flight during this pass
            const int in = (rb + gridDim.x) * RP + rl;
#pragma unroll
            for (int a = 0; a < D; ++a) xn[a] = in < n ? x[(long)in * D + a] : (T)0;
        }
        // every wave holds the same rows, so this choice is the workgroup's
        const bool exact = bad || __any(rbad);
        T v = -R::inf(), rv = -R::inf();   // best and (FLAGS) runner-up
        int jb = 0x7fffffff;
        if (!exact) {
            T best = -R::inf(), other = -R::inf();   // other: the other tiles' maxima
            int bt = -1;
            for (int tt = 0; tt < span && jw0 + tt < n_prev; tt += kTile) {
                T c[kRowsPer];
                row_edge_scores<T, D, kRowsPer, kTile>(tw + (long)tt * (D + 1), y, c);
                T mx = vmax_(vmax_(c[0], c[1]), c[2]);
#pragma unroll
                for (int k = 3; k + 1 < kRowsPer; k += 2) mx = vmax_(vmax_(mx, c[k]), c[k + 1]);
                if (kRowsPer % 2 == 0) mx = vmax_(mx, c[kRowsPer - 1]);
                const bool up = mx > best;
                if (FLAGS) other = up ? best : vmax_(other, mx);
                bt = up ? tt : bt;
                best = up ? mx : best;
            }
            rv = other;
            if (bt >= 0) {
                T c[kRowsPer];
                row_edge_scores<T, D, kRowsPer, kTile>(tw + (long)bt * (D + 1), y, c);
#pragma unroll
                for (int k = 0; k < kRowsPer; ++k) {
                    const bool b = c[k] > v;
                    v = b ? c[k] : v;
                    jb = b ? jw + bt + k : jb;
                }
                if (FLAGS) {
#pragma unroll
                    for (int k = 0; k < kRowsPer; ++k) rv = jw + bt + k == jb ? rv : vmax_(rv, c[k]);
                }
            }
        } else {
            for (int tt = 0; tt < span && jw + tt < n_prev; tt += kTile) {
                T c[kRowsPer];
                row_edge_scores<T, D, kRowsPer, kTile>(tw + (long)tt * (D + 1), y, c);
#pragma unroll
                for (int k = 0; k < kRowsPer; ++k) {
                    const int j = jw + tt + k;
                    if (j < n_prev) {
                        nan_seen |= live && (c[k] != c[k]);
                        const bool b = c[k] > v;
                        if (FLAGS) rv = b ? v : (c[k] > rv ? c[k] : rv);
                        v = b ? c[k] : v;
                        jb = b ? j : jb;
                    }
                }
            }
        }
#pragma unroll
        for (int off = RP; off < kWave; off <<= 1) {
            const T vo = __shfl_xor(v, off, kWave);
            const int jo = __shfl_xor(jb, off, kWave);
            if (FLAGS) take_better(v, jb, rv, vo, jo, __shfl_xor(rv, off, kWave));
            else take_better(v, jb, vo, jo);
        }
        if (lane < RP) {
            s_v[w][lane] = v;
            s_j[w][lane] = jb;
            if (FLAGS) s_r[FLAGS ? w : 0][lane] = rv;
        }
        __syncthreads();
        if (w == 0) {
            // the 16 waves' results of row rl: lane group grp takes waves
            // grp, grp + 64 / RP, ..., then the groups merge by shuffles
            constexpr int kGroups = kWave / RP;
            T b = s_v[grp][rl];
            int arg = s_j[grp][rl];
            T r = FLAGS ? s_r[FLAGS ? grp : 0][rl] : (T)0;
#pragma unroll
            for (int q = 1; q < kRowsWaves / kGroups; ++q) {
                const int h = grp + q * kGroups;
                if (FLAGS) take_better(b, arg, r, s_v[h][rl], s_j[h][rl], s_r[FLAGS ? h : 0][rl]);
                else take_better(b, arg, s_v[h][rl], s_j[h][rl]);
            }
#pragma unroll
            for (int off = RP; off < kWave; off <<= 1) {
                const T vo = __shfl_xor(b, off, kWave);
                const int jo = __shfl_xor(arg, off, kWave);
                if (FLAGS) take_better(b, arg, r, vo, jo, __shfl_xor(r, off, kWave));
                else take_better(b, arg, vo, jo);
            }
            if (lane < RP && live) {
                const T ell = F::loglik(m, s_z, mk, xi);
                const T ph = b * (T)kLn2 + ell;
                phi[i] = ph;
                psi[i] = arg == 0x7fffffff ? 0 : arg;
                if (FLAGS) {
                    // runner-up within tie_tol max(1, |best|), in log2 units
                    const T mag = b < 0 ? -b : b;
                    const T sc = mag > (T)kLog2e ? mag : (T)kLog2e;
                    flags[i] = (n_prev > 1 && r >= b - tie_tol * sc) ? 1 : 0;
                }
                nan_seen |= (ell != ell) || (ph != ph);
            }
        }
        __syncthreads();
    }
    if (__any(nan_seen) && lane == 0) atomicOr(status, STATUS_NONFINITE);
}

// ---------------------------------------------------------------------------
// Backtracking: one workgroup (one wave) per sequence.
// ---------------------------------------------------------------------------
// One sequence with a particle count per step: cnt [T + 1] (cnt[0] = 1),
// psi rows of stride n_max; i_T = lowest argmax of phi_T over cnt[T].
template <typename T>
__global__ __launch_bounds__(64) void k_backtrack_steps(int T_, const int *__restrict__ cnt, int n_max,
                                                        const int32_t *__restrict__ psi,
                                                        const T *__restrict__ phi_T, int32_t *idx,
                                                        T *logpost, uint32_t *status)
{
    using R = RealOps<T>;
    const int lane = threadIdx.x;
    const int n = cnt[T_];
    ArgBest<T> ab{-R::inf(), -R::inf(), 0x7fffffff};   // the same reduction as k_backtrack
    for (int i = lane; i < n; i += kWave) {
        const T v = phi_T[i];
        if (i == lane) { ab.best = v; ab.arg = i; }
        else argbest_push(ab, v, i);
    }
    ab = wave_argbest(ab);
    if (lane != 0) return;
    const T best = ab.best;
    int cur = ab.arg;
    idx[T_ - 1] = cur;
    for (int t = T_; t >= 2; --t) {
        int prev = psi[(long)(t - 1) * n_max + cur];
        if (prev < 0 || prev >= cnt[t - 1]) { atomicOr(status, STATUS_NONFINITE); prev = 0; }
        idx[t - 2] = prev;
        cur = prev;
    }
    logpost[0] = best;
    if (!R::finite(best)) atomicOr(status, STATUS_NONFINITE);
}

template <typename T>
__global__ __launch_bounds__(64) void k_backtrack(int T_, int n, int d, const int32_t *__restrict__ psi,
                                                  long psi_bstride, const T *__restrict__ phi_T,
                                                  long phi_bstride, int32_t *idx_out, T *logpost,
                                                  const T *__restrict__ parts, long parts_bstride,
                                                  const T *__restrict__ x0, T *xmap, uint32_t *status)
{
    using R = RealOps<T>;
    const int b = blockIdx.x;
    const int lane = threadIdx.x;
    const T *ph = phi_T + (long)b * phi_bstride;
    ArgBest<T> ab{-R::inf(), -R::inf(), 0x7fffffff};
    for (int i = lane; i < n; i += kWave) {
        const T v = ph[i];
        if (i == lane) { ab.best = v; ab.arg = i; }
        else argbest_push(ab, v, i);
    }
    ab = wave_argbest(ab);
    int32_t *idx = idx_out + (long)b * T_;
    if (lane == 0) {
        int cur = ab.arg;
        idx[T_ - 1] = cur;
        const int32_t *ps = psi + (long)b * psi_bstride;
        for (int t = T_; t >= 2; --t) {
            int prev = ps[(long)(t - 1) * n + cur];
            if (prev < 0 || prev >= n) { atomicOr(status, STATUS_NONFINITE); prev = 0; }
            idx[t - 2] = prev;
            cur = prev;
        }
        logpost[b] = ab.best;
        if (!R::finite(ab.best)) atomicOr(status, STATUS_NONFINITE);
    }
    if (xmap == nullptr) return;
    __syncthreads();
    T *xm = xmap + (long)b * (T_ + 1) * d;
    for (int c = lane; c < d; c += kWave) xm[c] = x0[(long)b * d + c];
    const T *pb = parts + (long)b * parts_bstride;
    for (int q = lane; q < T_ * d; q += kWave) {
        const int t = q / d, c = q % d;
        xm[(long)(t + 1) * d + c] = pb[((long)t * n + idx[t]) * d + c];
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

} // namespace smsq
