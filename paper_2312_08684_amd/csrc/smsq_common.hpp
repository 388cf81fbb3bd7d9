// Device-side helpers shared by the Stein-MAP-Seq kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smsq {

constexpr int kWave = 64;
constexpr double kLog2e = 1.4426950408889634073599;
constexpr double kLn2 = 0.6931471805599453094172;
constexpr double kPi = 3.14159265358979323846;

// Padded row length of a d-dimensional particle in LDS: rows of 1, 2, 4 or 8
// elements so that a row is read with one or two aligned vector loads.
__host__ __device__ constexpr int dpad(int d) { return d <= 1 ? 1 : d <= 2 ? 2 : d <= 4 ? 4 : d <= 8 ? 8 : 16; }

// ---- real-type dispatch -----------------------------------------------------
template <typename T> struct RealOps;

template <> struct RealOps<float> {
    static __device__ __forceinline__ float exp2_(float x) { return __builtin_amdgcn_exp2f(x); }
    static __device__ __forceinline__ float exp_(float x) { return __expf(x); }
    static __device__ __forceinline__ float log_(float x) { return __logf(x); }
    static __device__ __forceinline__ float sqrt_(float x) { return __fsqrt_rn(x); }
    static __device__ __forceinline__ void sincos_(float x, float *s, float *c) { sincosf(x, s, c); }
    static __device__ __forceinline__ float atan2_(float y, float x) { return atan2f(y, x); }
    static __device__ __forceinline__ float floor_(float x) { return floorf(x); }
    static __device__ __forceinline__ float inf() { return __builtin_huge_valf(); }
    static __device__ __forceinline__ bool finite(float x) { return __builtin_isfinite(x); }
};

template <> struct RealOps<double> {
    static __device__ __forceinline__ double exp2_(double x) { return exp2(x); }
    static __device__ __forceinline__ double exp_(double x) { return exp(x); }
    static __device__ __forceinline__ double log_(double x) { return log(x); }
    static __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
    static __device__ __forceinline__ void sincos_(double x, double *s, double *c) { sincos(x, s, c); }
    static __device__ __forceinline__ double atan2_(double y, double x) { return atan2(y, x); }
    static __device__ __forceinline__ double floor_(double x) { return floor(x); }
    static __device__ __forceinline__ double inf() { return __builtin_huge_val(); }
    static __device__ __forceinline__ bool finite(double x) { return __builtin_isfinite(x); }
};

// Order-preserving unsigned key of a non-negative float / double (its bit
// pattern), used for exact order statistics by radix selection.
template <typename T> struct KeyOf;
template <> struct KeyOf<float> {
    using K = uint32_t;
    static constexpr int kPasses = 3;
    static __device__ __forceinline__ K key(float v) { return __float_as_uint(v); }
    static __device__ __forceinline__ float val(K k) { return __uint_as_float(k); }
    static __device__ __forceinline__ int shift(int p) { return p == 0 ? 21 : p == 1 ? 10 : 0; }
    static __device__ __forceinline__ int width(int p) { return p == 2 ? 10 : 11; }
};
template <> struct KeyOf<double> {
    using K = uint64_t;
    static constexpr int kPasses = 6;
    static __device__ __forceinline__ K key(double v) { return (K)__double_as_longlong(v); }
    static __device__ __forceinline__ double val(K k) { return __longlong_as_double((long long)k); }
    static __device__ __forceinline__ int shift(int p) { return p < 5 ? 53 - 11 * p : 0; }
    static __device__ __forceinline__ int width(int p) { return p < 5 ? 11 : 9; }
};

// ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a = 0xD2511F53u * c.x;
        const uint32_t ah = __umulhi(0xD2511F53u, c.x);
        const uint32_t b = 0xCD9E8D57u * c.z;
        const uint32_t bh = __umulhi(0xCD9E8D57u, c.z);
        U4 n;
        n.x = bh ^ c.y ^ k0;
        n.y = b;
        n.z = ah ^ c.w ^ k1;
        n.w = a;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// D standard normals (D <= 16) for (seed, sequence, step, particle): counter
// (i, t, seq, block) for blocks 0, 1, ... (four uniforms each, as many as
// the D/2 Box-Muller pairs need), uniforms (u + 0.5) 2^-32, Box-Muller in
// double precision.  The first eight normals do not depend on D.
template <int D>
__device__ inline void normals(uint64_t seed, uint32_t seq, uint32_t t, uint32_t i, double (&out)[D])
{
    static_assert(D >= 1 && D <= 16, "up to 16 normals");
    constexpr int kBlocks = (D + 3) / 4;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    double u[4 * kBlocks];
#pragma unroll
    for (int blk = 0; blk < kBlocks; ++blk) {
        U4 r = philox4x32_10(U4{i, t, seq, (uint32_t)blk}, k0, k1);
        u[4 * blk + 0] = ((double)r.x + 0.5) * (1.0 / 4294967296.0);
        u[4 * blk + 1] = ((double)r.y + 0.5) * (1.0 / 4294967296.0);
        u[4 * blk + 2] = ((double)r.z + 0.5) * (1.0 / 4294967296.0);
        u[4 * blk + 3] = ((double)r.w + 0.5) * (1.0 / 4294967296.0);
    }
#pragma unroll
    for (int p = 0; 2 * p < D; ++p) {
        const double rad = sqrt(-2.0 * log(u[2 * p]));
        double s, c;
        sincos(2.0 * kPi * u[2 * p + 1], &s, &c);
        out[2 * p] = rad * c;
        if (2 * p + 1 < D) out[2 * p + 1] = rad * s;
    }
}

// Index of the calling wave in its workgroup, as a scalar (wave-uniform)
// value so that loops over per-wave work compile to scalar loop control.
__device__ __forceinline__ int wave_id()
{
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
}

// ---- wave-level reductions ---------------------------------------------------
template <typename T> __device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane)
{
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t o = __shfl_up(v, off, kWave);
        if (lane >= off) v += o;
    }
    return v;
}

// (value, index, runner-up) triple for a max-plus row reduction: the lowest
// index among equal maxima wins; `second` is the best value among the other
// indices.
template <typename T> struct ArgBest {
    T best;
    T second;
    int arg;
};

template <typename T> __device__ __forceinline__ void argbest_push(ArgBest<T> &a, T c, int j)
{
    if (c > a.best) {
        a.second = a.best;
        a.best = c;
        a.arg = j;
    } else if (c > a.second) {
        a.second = c;
    }
}

template <typename T> __device__ __forceinline__ ArgBest<T> argbest_merge(ArgBest<T> a, ArgBest<T> b)
{
    // Winner: larger best, ties to the lower index.  Runner-up: the better of
    // the winner's runner-up and the loser's best.
    const bool b_wins = (b.best > a.best) || (b.best == a.best && b.arg < a.arg);
    ArgBest<T> w = b_wins ? b : a;
    ArgBest<T> l = b_wins ? a : b;
    w.second = w.second > l.best ? w.second : l.best;
    return w;
}

template <typename T> __device__ __forceinline__ ArgBest<T> wave_argbest(ArgBest<T> a)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        ArgBest<T> o;
        o.best = __shfl_xor(a.best, off, kWave);
        o.second = __shfl_xor(a.second, off, kWave);
        o.arg = __shfl_xor(a.arg, off, kWave);
        a = argbest_merge(a, o);
    }
    return a;
}

} // namespace smsq
