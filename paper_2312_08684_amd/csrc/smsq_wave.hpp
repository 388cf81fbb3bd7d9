// One-wave step kernel for small particle sets (n <= 64 and n_prev <= 64),
// the sizes of the paper's own experiments (N_s = 10..40).  The same time
// step as k_step (initial particles, L SVGD iterations with the median
// bandwidth, the score under the transition mixture and the Stein update,
// then the forward-recursion row of every particle), laid out for a single
// wave: lane i holds particle i and lane j the transition mean of previous
// particle j, in registers, and the loops over the other particles read them
// with readlane broadcasts instead of LDS round trips.  LDS holds only the
// n(n-1)/2 pair distances for the median, written to slot k(k-1)/2 + i and
// selected by the ballot bisection of the vector-ALU kernel.
#pragma once

#include "smsq_kernels.hpp"

namespace smsq {

constexpr int kWaveMaxParticles = 64;

template <typename T> __device__ __forceinline__ T lane_bcast(T v, int j);
template <> __device__ __forceinline__ float lane_bcast<float>(float v, int j)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}
template <> __device__ __forceinline__ double lane_bcast<double>(double v, int j)
{
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), j);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), j);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

template <typename T, int KIND, int D>
__global__ __launch_bounds__(64) void k_step_wave(StepArgs<T> a)
{
    using F = Family<T, KIND, D>;
    using R = RealOps<T>;
    using KO = KeyOf<T>;
    __shared__ T pairs[kWaveMaxParticles * (kWaveMaxParticles - 1) / 2];
    const int b = blockIdx.x;
    const int lane = threadIdx.x;
    const int n = a.n, np = a.n_prev;
    const DevModel<T> &m = a.m;
    const T *xprev = a.x_prev + (long)b * a.x_prev_stride;
    T *xg = a.x + (long)b * a.x_stride;
    const T *z = a.z + (long)b * a.z_stride;
    const uint8_t *mk = a.mask ? a.mask + (long)b * a.mask_stride : nullptr;

    // particles and means relative to the first previous particle's
    // transition mean, as in k_step
    T cen[D], rs[D];
    {
        T xp[D];
#pragma unroll
        for (int c = 0; c < D; ++c) xp[c] = xprev[c];
        F::mean(m, a.t, xp, cen);
    }
#pragma unroll
    for (int c = 0; c < D; ++c) rs[c] = m.rs[c];
    // lane j: the centred mean scaled to log2 units and the log2-weight
    T mj[D], cj = -R::inf();
#pragma unroll
    for (int c = 0; c < D; ++c) mj[c] = (T)0;
    if (lane < np) {
        T xp[D], mu[D];
#pragma unroll
        for (int c = 0; c < D; ++c) xp[c] = xprev[(long)lane * D + c];
        F::mean(m, a.t, xp, mu);
#pragma unroll
        for (int c = 0; c < D; ++c) mj[c] = (mu[c] - cen[c]) * rs[c];
        const T lw = a.log_w ? a.log_w[(long)b * a.log_w_stride + lane] : -R::log_((T)np);
        cj = lw * (T)kLog2e;
    }
    // lane i: its particle, centred
    T xi[D];
#pragma unroll
    for (int c = 0; c < D; ++c) xi[c] = (T)0;
    if (lane < n) {
        if (a.init_given) {
#pragma unroll
            for (int c = 0; c < D; ++c) xi[c] = xg[(long)lane * D + c] - cen[c];
        } else {
            T xp[D], mu[D];
            const int j = lane % np;
#pragma unroll
            for (int c = 0; c < D; ++c) xp[c] = xprev[(long)j * D + c];
            F::mean(m, a.t, xp, mu);
            double nz[D];
            normals<D>(a.seed, a.seq_offset + (uint32_t)b, (uint32_t)a.t, (uint32_t)lane, nz);
#pragma unroll
            for (int c = 0; c < D; ++c) xi[c] = (mu[c] - cen[c]) + m.sqrt_q[c] * (T)nz[c];
        }
    }
    // mean of the transition means (paper-literal score reading)
    T mbar_all[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
        const T v = lane < np ? mj[c] / rs[c] : (T)0;
        mbar_all[c] = wave_sum(v) / (T)np;
    }

    const uint32_t M = (uint32_t)(n * (n - 1) / 2);
    const T inv_n = (T)1 / (T)n;
    T h = (T)1;
    for (int it = 0; a.do_svgd && it < a.n_iter; ++it) {
        // (1) bandwidth: all pair distances to LDS, exact lower median
        if (a.bw_mode == 0 || it == 0) {
            T med = (T)0;
            if (M > 0) {
                // four columns at a time: independent chains for one wave
                int k = 1;
                for (; k + 4 <= n; k += 4) {
                    T dd[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        dd[u] = 0;
#pragma unroll
                        for (int c = 0; c < D; ++c) {
                            const T r = xi[c] - lane_bcast(xi[c], k + u);
                            dd[u] += r * r;
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (lane < k + u) pairs[(uint32_t)((k + u) * (k + u - 1) / 2 + lane)] = dd[u];
                }
                for (; k < n; ++k) {
                    T dd = 0;
#pragma unroll
                    for (int c = 0; c < D; ++c) {
                        const T r = xi[c] - lane_bcast(xi[c], k);
                        dd += r * r;
                    }
                    if (lane < k) pairs[(uint32_t)(k * (k - 1) / 2 + lane)] = dd;
                }
                __syncthreads();
                const uint32_t rank = (M - 1) / 2;
                const uint32_t used = (M + kWave - 1) / kWave;
                typename KO::K key;
                if (used <= 1) key = select_rank_wave<T, 1>(pairs, M, rank, lane);
                else if (used <= 2) key = select_rank_wave<T, 2>(pairs, M, rank, lane);
                else if (used <= 4) key = select_rank_wave<T, 4>(pairs, M, rank, lane);
                else if (used <= 8) key = select_rank_wave<T, 8>(pairs, M, rank, lane);
                else if (used <= 16) key = select_rank_wave<T, 16>(pairs, M, rank, lane);
                else key = select_rank_wave<T, 32>(pairs, M, rank, lane);
                med = KO::val(key);
                __syncthreads();
            }
            h = bandwidth_from_median(med, n, a.bw_scale);
        }
        if (a.h_out && lane == 0) a.h_out[(long)b * a.h_stride + it] = h;

        // (2) score of lane i's particle
        T sk[D];
        {
            T g[D], mb[D];
#pragma unroll
            for (int c = 0; c < D; ++c) g[c] = (T)0;
            if (lane < n) {
                T xa[D];
#pragma unroll
                for (int c = 0; c < D; ++c) xa[c] = xi[c] + cen[c];
                F::grad(m, z, mk, xa, g);
            }
            if (a.trans_mode == 0) {
                T xs[D];
#pragma unroll
                for (int c = 0; c < D; ++c) xs[c] = xi[c] * rs[c];
                T mx = -R::inf(), sum = 0, acc[D];
#pragma unroll
                for (int c = 0; c < D; ++c) acc[c] = (T)0;
                constexpr int CH = 4;
                int j0 = 0;
                for (; j0 + CH <= np; j0 += CH) {
                    T av[CH], mv[CH][D];
#pragma unroll
                    for (int u = 0; u < CH; ++u) {
                        T q2 = 0;
#pragma unroll
                        for (int c = 0; c < D; ++c) {
                            mv[u][c] = lane_bcast(mj[c], j0 + u);
                            const T r = xs[c] - mv[u][c];
                            q2 += r * r;
                        }
                        av[u] = lane_bcast(cj, j0 + u) - q2;
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
#pragma unroll
                        for (int c = 0; c < D; ++c) acc[c] += e * mv[u][c];
                    }
                }
                for (; j0 < np; ++j0) {
                    T mv[D], q2 = 0;
#pragma unroll
                    for (int c = 0; c < D; ++c) {
                        mv[c] = lane_bcast(mj[c], j0);
                        const T r = xs[c] - mv[c];
                        q2 += r * r;
                    }
                    const T av = lane_bcast(cj, j0) - q2;
                    const T nm = av > mx ? av : mx;
                    const T sf = R::exp2_(mx - nm);
                    const T e = R::exp2_(av - nm);
                    sum = sum * sf + e;
#pragma unroll
                    for (int c = 0; c < D; ++c) acc[c] = acc[c] * sf + e * mv[c];
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
            for (int c = 0; c < D; ++c) sk[c] = lane < n ? g[c] - (xi[c] - mb[c]) * m.inv_q[c] : (T)0;
        }

        // (3) Stein direction and synchronous update
        const T beta = (T)kLog2e / h;
        const T c2 = (T)2 / h;
        const T inv_h = (T)1 / h;
        T as[D], ar[D];
#pragma unroll
        for (int c = 0; c < D; ++c) { as[c] = 0; ar[c] = 0; }
        // four sources at a time (independent chains), summed in order
        auto pair_terms = [&](int k, T (&df)[D], T (&skb)[D], T &kap, T &w) {
            T dd = 0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                df[c] = xi[c] - lane_bcast(xi[c], k);
                skb[c] = lane_bcast(sk[c], k);
                dd += df[c] * df[c];
            }
            if (a.kernel == 0) {
                kap = R::exp2_(-beta * dd);
                w = kap;  // times 2/h below
            } else {
                stein_kernel<T>(a.kernel, dd, inv_h, kap, w);
            }
        };
        int k = 0;
        for (; k + 4 <= n; k += 4) {
            T df[4][D], skb[4][D], kap[4], w[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) pair_terms(k + u, df[u], skb[u], kap[u], w[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int c = 0; c < D; ++c) { as[c] += kap[u] * skb[u][c]; ar[c] += w[u] * df[u][c]; }
        }
        for (; k < n; ++k) {
            T df[D], skb[D], kap, w;
            pair_terms(k, df, skb, kap, w);
#pragma unroll
            for (int c = 0; c < D; ++c) { as[c] += kap * skb[c]; ar[c] += w * df[c]; }
        }
        const T cw = a.kernel == 0 ? c2 : (T)1;
        if (lane < n) {
#pragma unroll
            for (int c = 0; c < D; ++c) xi[c] += a.step * ((as[c] + cw * ar[c]) * inv_n);
        }
    }

    // write particles back; flag non-finite values
    bool bad = false;
    if (a.do_svgd && lane < n) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const T v = xi[c] + cen[c];
            bad |= !R::finite(v);
            xg[(long)lane * D + c] = v;
        }
    }

    if (a.do_viterbi) {
        // forward recursion: c_ij = log_z - ln2 |xs_i - ms_j|^2 + phi_prev(j)
        const T pj = (lane < np && a.phi_prev) ? a.phi_prev[(long)b * a.phi_prev_stride + lane] : (T)0;
        T xs[D];
#pragma unroll
        for (int c = 0; c < D; ++c) xs[c] = xi[c] * rs[c];
        ArgBest<T> ab{-R::inf(), -R::inf(), 0};
        bool nan_seen = false;
        for (int j = 0; j < np; ++j) {
            T q2 = 0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const T r = xs[c] - lane_bcast(mj[c], j);
                q2 += r * r;
            }
            const T A = m.log_z - (T)kLn2 * q2;
            const T cij = A + lane_bcast(pj, j);
            nan_seen |= (cij != cij);
            if (j == 0) { ab.best = cij; ab.arg = 0; }
            else argbest_push(ab, cij, j);
        }
        if (lane < n) {
            T xa[D];
#pragma unroll
            for (int c = 0; c < D; ++c) xa[c] = xi[c] + cen[c];
            const T ell = F::loglik(m, z, mk, xa);
            const T ph = ab.best + ell;
            nan_seen |= (ph != ph);
            bad |= nan_seen;
            a.phi[(long)b * a.phi_stride + lane] = ph;
            a.psi[(long)b * a.psi_stride + lane] = ab.arg;
            if (a.flags) {
                const T sc_ = ab.best > (T)1 || ab.best < (T)-1 ? (ab.best < 0 ? -ab.best : ab.best) : (T)1;
                a.flags[(long)b * a.flags_stride + lane] =
                    (np > 1 && ab.second >= ab.best - a.tie_tol * sc_) ? 1 : 0;
            }
        }
    }
    if (__any(bad) && lane == 0) atomicOr(a.status, STATUS_NONFINITE);
}

} // namespace smsq
