// FP32 step kernel on the matrix cores (v_mfma_f32_16x16x4f32 and
// v_mfma_f32_4x4x1f32, wave64).
//
// Same computation as k_step (one workgroup per sequence, state in LDS), with
// the pairwise work of every SVGD iteration (eq. SVGD_newupdate) on MFMA:
//   * bandwidth: the squared distances D_ik = n_i + n_k - 2 x_i . x_k come
//     from 16x16 Gram tiles; the exact lower median is found by one pass that
//     counts the distances below a window predicted from the previous
//     iterations' medians and keeps (and bins) those inside it, then a rank
//     among the kept values of the median's bin (radix selections as
//     fallbacks);
//   * scores: the transition-mixture softmax over the previous particles,
//     logit_kj = 2 mh_j . xh_k + c_j - |mh_j|^2 (log2 units; the common
//     -|xh_k|^2 drops out), as 16x16 logit tiles [xh_k, 1] . [2 mh_j, c'_j],
//     a per-particle reference maximum raised only when a tile exceeds it by
//     2^64, exp2 on the VALU, and the weighted sums sum_j e_kj [2 mh_j, 1]
//     accumulated by MFMA;
//   * Stein direction: Gram tiles give the kernel argument
//     2 beta x_k . x_i - beta n_k (the norm rides in the free eighth
//     K-column), kappa_ik = exp2(that - beta n_i) with beta = log2(e) / h,
//     and sum_k kappa_ik [s_k - (2/h) x_k, 1] is accumulated by MFMA.
// Particles are stored centred on the mean of the previous step's transition
// means, which keeps |x|^2 small next to the squared distances in FP32.
//
// Operand layouts of v_mfma_f32_16x16x4f32 (checked on gfx950): lane l gives
// A[l % 16][l / 16] and B[l / 16][l % 16]; result register r of lane l is
// D[4 (l / 16) + r][l % 16].
#pragma once

#include "smsq_kernels.hpp"

namespace smsq {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float fmax_(float a, float b) { return a > b ? a : b; }

// a block-uniform value kept in a scalar register
__device__ __forceinline__ float uniform(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ uint32_t lanes_below(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Lanes of the diagonal 16x16 distance tile that hold a pair k > i in
// result register r (k = 4 (l / 16) + r, i = l % 16).
__host__ __device__ constexpr unsigned long long diag_lanes(int r)
{
    unsigned long long m = 0;
    for (int l = 0; l < 64; ++l)
        if (4 * (l >> 4) + r > (l & 15)) m |= 1ull << l;
    return m;
}

// max over the four 16-lane groups that hold the same column (lanes l, l^16,
// l^32, l^48)
__device__ __forceinline__ float group_max4(float v)
{
    auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    const float m1 = fmax_(__uint_as_float(a[0]), __uint_as_float(a[1]));
    auto b = __builtin_amdgcn_permlane16_swap(__float_as_uint(m1), __float_as_uint(m1), false, false);
    return fmax_(__uint_as_float(b[0]), __uint_as_float(b[1]));
}

// Up to sixteen waves per workgroup (four per SIMD), one 64-particle task
// each at the largest size.
constexpr int kMaxWaves = 16;
constexpr int kTilesPerWave = 4;  // register blocking: 64 particles per wave task
constexpr int kMaxParticles = 1024;  // largest sequence the kernel takes
// A workgroup of W waves takes up to W * TS tasks (TS task slots per wave).
constexpr int kVtRows = 9;        // rows of the transition-mean table: 2 mh (7), 1, c'
constexpr int kWinCap = 8192;     // capacity of the median window buffer (floats)
constexpr int kWinRegion = kWinCap / kMaxWaves; // per-wave share of the window buffer
constexpr int kWinTarget = 512;   // aimed-for number of distances in the window
// log2 headroom before the softmax reference moves: a tile's exponentials
// stay at most 2^64 and a row's sums of up to 1024 of them far below the
// FP32 range, while a column's reference seldom moves after its first tile
constexpr float kRescaleGap = 64.f;
constexpr int kProgSlot = 48;      // first of the 16 wave-progress words in the reduction slots
constexpr int kPartStride = 9;     // floats per particle in a split's partial sums (8 rows + 1)

// LDS byte layout of the MFMA step workgroup, and how its waves share the
// pairwise work.  With fewer 64-particle tasks than waves (N below 1024 for
// 16 waves) the source tiles of each task are split among several waves
// ("splits"): a wave handles task w % ntasks over the split w / ntasks of
// the source range, leaves partial sums in LDS, and the partials are merged
// in split order (the same result whatever the timing).  ns_sc / ns_st are
// the splits of the score and Stein passes (at most the source tiles each
// pass has); nwaves the waves a launch of this shape uses.
// A workgroup of the multi-workgroup mode owns tasks_local of the tasks (its
// targets) and holds every particle; win_cap is its window buffer's capacity.
struct MfmaLds {
    long off_x, off_s, off_m, off_phip, off_scr, off_win, off_z, off_mask, off_red, off_part, total;
    int npad, nppad, nwaves, ntasks, ns_sc, ns_st, ns_max, win_cap, win_region;
    __host__ __device__ MfmaLds(int n, int n_prev, int waves = kMaxWaves, int tasks_local = 0,
                                int win = kWinCap)
    {
        npad = (n + 63) / 64 * 64;
        nppad = (n_prev + 15) / 16 * 16;
        ntasks = tasks_local > 0 ? tasks_local : npad / 64;
        win_cap = win;
        win_region = win / kMaxWaves;
        if (ntasks >= waves) {
            ns_sc = ns_st = ns_max = 1;
            nwaves = waves;
        } else {
            const int cap = waves / ntasks;
            ns_sc = cap < nppad / 16 ? cap : nppad / 16;
            ns_st = cap < npad / 16 ? cap : npad / 16;
            ns_max = ns_sc > ns_st ? ns_sc : ns_st;
            nwaves = ntasks * ns_max;
        }
        long o = 0;
        off_x = o; o += align16((long)npad * 8 * 4);
        off_s = o; o += align16((long)npad * 8 * 4);
        off_m = o; o += align16((long)kVtRows * nppad * 4);
        off_phip = o; o += align16((long)nppad * 4);
        off_scr = o; o += (long)kBins * 4;  // the radix-selection histogram
        off_win = o; o += (long)(win_cap + 256) * 4;       // window buffer + its histogram
        off_z = o; o += align16((long)kMaxObs * 4);
        off_mask = o; o += 64;
        off_red = o; o += 512;  // uint slots 0..63 (48..63: wave progress), float slots from byte 256
        // partial sums of the splits: [ns_max][ntasks * 64][9] floats
        off_part = o; o += ns_max > 1 ? align16((long)ns_max * ntasks * 64 * kPartStride * 4) : 0;
        total = o;
    }
};

// K-chunks of the distance and Gram tiles.  Eight K-rows (two MFMAs) hold
// up to seven coordinates and the norm in row 7; with K4 (d <= 3) four
// K-rows (one MFMA) hold up to three coordinates and the norm in row 3.
// ka(g): the particle-row column that K-row g (of the first chunk) reads.
template <bool K4> __device__ __forceinline__ int gram_col(int g) { return K4 && g == 3 ? 7 : g; }

// Visits the squared distances D_ik = n_i + n_k - 2 x_i . x_k of every pair
// i < k from 16x16 MFMA Gram tiles: the A rows are the source particles with
// their norm n_k in the last K-row (coordinates zero-padded), the B columns
// are -2 x_i with a 1 in that row, and the accumulator starts at n_i, so
// the tile holds the distances themselves.  Each wave takes whole rows of tiles
// (target tile ib, source tiles kb >= ib) and issues the MFMAs of four source
// tiles before using any result.  fn(Dv, diag) receives the four distances
// of a lane for one tile (k = 16 kb + 4 g + r, i = 16 ib + col); in the
// diagonal tile (diag true) only the lanes of diag_lanes(r) hold pairs k > i.
// Pad particles have n = +inf, so their distances are +inf.  The median
// window pass (TileWalker) computes every distance the same way.
template <bool K4, typename Fn>
__device__ __forceinline__ void for_each_distance(const float *X8, int npad, Fn &&fn, int vwave = -1, int nvwaves = 0)
{
    constexpr int kBatch = 4;
    const int lane = threadIdx.x & 63;
    const int wave = nvwaves > 0 ? vwave : wave_id(), nwaves = nvwaves > 0 ? nvwaves : (int)(blockDim.x >> 6);
    const int g = lane >> 4, col = lane & 15;
    const int nt16 = npad / 16;
    // Rows of tiles (target tile ib, source tiles kb >= ib) go to the waves in
    // snake order, which gives every wave the same number of tiles when the
    // row count is a multiple of 2 * nwaves.
    for (int rr = 0;; ++rr) {
        const int ib = (rr & 1) ? (rr + 1) * nwaves - 1 - wave : rr * nwaves + wave;
        if (ib >= nt16) break;
        const int i0 = ib * 16;
        const float *xi = X8 + (long)(i0 + col) * 8;
        const int ka = gram_col<K4>(g);
        const float bi0 = K4 && g == 3 ? 1.f : -2.f * xi[g];
        const float bi1 = g == 3 ? 1.f : -2.f * xi[4 + g];
        const float nni = xi[7];
        const f32x4 cn = {nni, nni, nni, nni};
        fn(K4 ? mfma16(xi[ka], bi0, cn) : mfma16(xi[4 + g], bi1, mfma16(xi[g], bi0, cn)), true);
        // A operands of a batch of source tiles; past the row's end a tile is
        // repeated and its results are not used
        float a0[kBatch], a1[kBatch];
        auto load_batch = [&](int kb) {
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const float *xk = X8 + (long)(min(kb + u, nt16 - 1) * 16 + col) * 8;
                a0[u] = xk[ka];
                a1[u] = K4 ? 0.f : xk[4 + g];
            }
        };
        load_batch(ib + 1);
        for (int kb = ib + 1; kb < nt16; kb += kBatch) {
            f32x4 G[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) G[u] = K4 ? mfma16(a0[u], bi0, cn) : mfma16(a1[u], bi1, mfma16(a0[u], bi0, cn));
            load_batch(kb + kBatch);  // next batch's loads overlap this batch's work
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                if (kb + u >= nt16) break;
                fn(G[u], false);
            }
        }
    }
}

// Exact order statistic `rank` of the squared distances by radix selection
// over the bit patterns (digits of 11, 11 and 10 bits); every pass recomputes
// the distances.  In diagonal tiles only pairs k > i count.
template <bool K4>
__device__ float radix_median_mfma(const float *X8, int npad, uint32_t rank, uint32_t *hist,
                                   uint32_t *red)
{
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = wave_id();
    uint32_t prefix = 0, pmask = 0;
    for (int pass = 0; pass < 3; ++pass) {
        const int shift = pass == 0 ? 21 : pass == 1 ? 10 : 0;
        const uint32_t dmask = pass == 2 ? 0x3ffu : 0x7ffu;
        for (int b = tid; b < kBins; b += nt) hist[b] = 0;
        __syncthreads();
        for_each_distance<K4>(X8, npad, [&](const f32x4 &Dv, bool diag) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t key = __float_as_uint(fmax_(Dv[r], 0.f));
                const bool valid = !diag || ((diag_lanes(r) >> lane) & 1ull);
                if (valid && (key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & dmask], 1u);
            }
        });
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
        prefix |= red[0] << shift;
        rank = red[1];
        pmask |= dmask << shift;
        __syncthreads();
    }
    return __uint_as_float(prefix);
}

// Exact order statistic r of the values kept in the window buffer: wave w's
// values sit in buf[w * kWinRegion ...] with wcnt[w] of them, all in
// [lo, hi) (key_lo, key_hi their bit patterns).  Radix selection on the key
// offsets key - key_lo, 8 bits per pass, as many passes as the span needs.
__device__ float buffer_select(const float *buf, const uint32_t *wcnt, int nregions, int region, uint32_t r,
                               uint32_t key_lo, uint32_t key_hi, uint32_t *hist, uint32_t *red)
{
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = wave_id();
    const uint32_t span = key_hi - key_lo;
    const int bits = span == 0 ? 1 : 32 - __clz(span);
    const int passes = (bits + 7) / 8;
    const int nslots = nregions * region;
    uint32_t prefix = 0, pmask = 0;
    for (int p = passes - 1; p >= 0; --p) {
        const int shift = 8 * p;
        for (int q = tid; q < 256; q += nt) hist[q] = 0;
        __syncthreads();
        for (int s = tid; s < nslots; s += nt) {
            if ((uint32_t)(s % region) < wcnt[s / region]) {
                const uint32_t k = __float_as_uint(buf[s]) - key_lo;
                if ((k & pmask) == prefix) atomicAdd(&hist[(k >> shift) & 0xffu], 1u);
            }
        }
        __syncthreads();
        if (wave == 0) {
            uint32_t c[4];
            uint32_t cnt = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) { c[q] = hist[lane * 4 + q]; cnt += c[q]; }
            const uint32_t incl = wave_incl_scan(cnt, lane);
            const uint32_t excl = incl - cnt;
            if (r >= excl && r < incl) {
                uint32_t rr = r - excl;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (rr < c[q]) { red[8] = (uint32_t)(lane * 4 + q); red[9] = rr; break; }
                    rr -= c[q];
                }
            }
        }
        __syncthreads();
        prefix |= red[8] << shift;
        r = red[9];
        pmask |= 0xffu << shift;
        __syncthreads();
    }
    return __uint_as_float(key_lo + prefix);
}

// Exact order statistic r of the values kept in the window buffer (same
// layout as buffer_select).  whist holds their histogram over 256 bins of
// (key - key_lo) >> shift, counted as the values were appended.  Wave 0
// finds the bin holding rank r; every wave gathers that bin's values from
// its own region into cand (positions from an LDS counter: the order does
// not matter); wave 0 ranks the candidates by comparison.  A bin with more
// than 64 values (heavy ties) falls back to buffer_select.  cand may alias
// whist: the histogram is dead once the bin is known.
__device__ float window_select(const float *buf, const uint32_t *wcnt, int nregions, int region, uint32_t r,
                               uint32_t key_lo, uint32_t key_hi, uint32_t shift, uint32_t *whist, uint32_t *red,
                               float *cand)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id(), nwaves = blockDim.x >> 6;
    if (wave == 0) {
        typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
        const u32x4_t c = *(const u32x4_t *)(whist + lane * 4);
        const uint32_t cnt = c[0] + c[1] + c[2] + c[3];
        const uint32_t incl = wave_incl_scan(cnt, lane);
        const uint32_t excl = incl - cnt;
        if (r >= excl && r < incl) {
            uint32_t rr = r - excl;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (rr < c[q]) {
                    red[2] = (uint32_t)(lane * 4 + q);
                    red[3] = rr;
                    red[4] = c[q];
                    break;
                }
                rr -= c[q];
            }
        }
        if (lane == 0) red[6] = 0;
    }
    __syncthreads();
    const uint32_t bin = red[2], rr = red[3], cb = red[4];
    if (cb > (uint32_t)kWave) return buffer_select(buf, wcnt, nregions, region, r, key_lo, key_hi, whist, red);
    for (int w = wave; w < nregions; w += nwaves) {
        const uint32_t c = wcnt[w];
        for (uint32_t s = lane; s < c; s += kWave) {
            const float v = buf[w * region + s];
            if (((__float_as_uint(v) - key_lo) >> shift) == bin) cand[atomicAdd(&red[6], 1u)] = v;
        }
    }
    __syncthreads();
    if (wave == 0 && (uint32_t)lane < cb) {
        const float v = cand[lane];
        uint32_t less = 0, leq = 0;
        for (uint32_t t = 0; t < cb; ++t) {
            const float u = cand[t];
            less += u < v ? 1u : 0u;
            leq += u <= v ? 1u : 0u;
        }
        if (less <= rr && rr < leq) red[5] = __float_as_uint(v);
    }
    __syncthreads();
    return __uint_as_float(red[5]);
}

// One wave's walk over its share of the off-diagonal distance tiles (the
// rows of tiles of for_each_distance, in the same order, source tiles
// kb > ib), two source tiles kb, kb + 1 per step.  Holds the current row's
// B operand (-2 x_i with a 1 in the norm row) and the target norms as the
// accumulator input.  The diagonal tiles of the wave's rows are visited by
// diagonals().  In chunk mode (the multi-workgroup walk: more waves than
// rows) virtual wave v of nv takes the v-th of nv equal contiguous runs of
// the off-diagonal tiles listed row by row, and every nv-th diagonal tile
// (CHUNK: the mode is fixed per kernel, so neither walk carries the other's
// state through its loops).
template <bool K4, bool CHUNK>
struct TileWalker {
    static constexpr bool chunk = CHUNK;
    int nt16, nwaves, wave, rr, ib, kb, left;
    float bi0, bi1;
    f32x4 cn;

    __device__ int row_of(int r) const { return (r & 1) ? (r + 1) * nwaves - 1 - wave : r * nwaves + wave; }
    __device__ void load_row(const float *X8, int g, int col)
    {
        const float *xi = X8 + (long)(ib * 16 + col) * 8;
        bi0 = K4 && g == 3 ? 1.f : -2.f * xi[g];
        bi1 = g == 3 ? 1.f : -2.f * xi[4 + g];
        const float nni = xi[7];
        cn = f32x4{nni, nni, nni, nni};
    }
    __device__ void start(const float *X8, int npad, int g, int col, int vwave = -1, int nvwaves = 0)
    {
        nt16 = npad / 16;
        nwaves = chunk ? nvwaves : (int)(blockDim.x >> 6);
        wave = chunk ? vwave : wave_id();
        if (!chunk) {
            left = 0x7fffffff;
            rr = -1;
            next_row(X8, g, col);
            return;
        }
        const long total = (long)nt16 * (nt16 - 1) / 2;
        long p0 = total * wave / nwaves;
        left = (int)(total * (wave + 1) / nwaves - p0);
        ib = 0;
        while (ib < nt16 - 1 && p0 >= nt16 - 1 - ib) {
            p0 -= nt16 - 1 - ib;
            ++ib;
        }
        kb = ib + 1 + (int)p0;
        if (left <= 0) ib = nt16;
        else load_row(X8, g, col);
    }
    // next row with an off-diagonal tile
    __device__ void next_row(const float *X8, int g, int col)
    {
        if (chunk) {
            ++ib;
            kb = ib + 1;
            if (left <= 0 || kb >= nt16) ib = nt16;
            else load_row(X8, g, col);
            return;
        }
        do {
            ++rr;
            ib = row_of(rr);
            kb = ib + 1;
        } while (ib < nt16 && kb >= nt16);
        if (ib < nt16) load_row(X8, g, col);
    }
    __device__ bool done() const { return ib >= nt16; }
    __device__ bool second() const { return kb + 1 < nt16 && left >= 2; }
    // distances of tiles kb and kb + 1 (clamped to the row: always in
    // bounds, also once the walk is done; results past the end are unused)
    __device__ void issue(const float *X8, int g, int col, f32x4 &D0, f32x4 &D1) const
    {
        const int k0 = min(kb, nt16 - 1), k1 = min(kb + 1, nt16 - 1);
        const float *x0 = X8 + (long)(k0 * 16 + col) * 8;
        const float *x1 = X8 + (long)(k1 * 16 + col) * 8;
        const int ka = gram_col<K4>(g);
        D0 = mfma16(x0[ka], bi0, cn);
        D1 = mfma16(x1[ka], bi0, cn);
        if (!K4) {
            D0 = mfma16(x0[4 + g], bi1, D0);
            D1 = mfma16(x1[4 + g], bi1, D1);
        }
    }
    __device__ void advance(const float *X8, int g, int col)
    {
        left -= second() ? 2 : 1;
        kb += 2;
        if (left <= 0) ib = nt16;
        else if (kb >= nt16) next_row(X8, g, col);
    }
    // the diagonal tile of every row of this wave (chunk mode: every
    // nwaves-th row), fn(D, true)
    template <typename Fn> __device__ void diagonals(const float *X8, int g, int col, Fn &&fn)
    {
        for (int r = 0;; ++r) {
            ib = chunk ? wave + r * nwaves : row_of(r);
            if (ib >= nt16) break;
            load_row(X8, g, col);
            const float *xk = X8 + (long)(ib * 16 + col) * 8;
            fn(K4 ? mfma16(xk[gram_col<K4>(g)], bi0, cn) : mfma16(xk[4 + g], bi1, mfma16(xk[g], bi0, cn)), true);
        }
    }
};

// Median tracker across the iterations of one step.  The previous two
// medians predict a window [lo, hi).  While the particles are unchanged (the
// score pass of the same iteration) the waves visit every distance once,
// counting those below lo and keeping those inside the window, each wave in
// its own region of the window buffer; finish() then selects the exact
// rank-th value among the kept ones.  When there is no prediction yet, the
// window misses the rank or a region overflows, the full radix selection
// runs instead.  Both read the same MFMA distances, so the result is the same
// exact lower median either way.
struct MedianTracker {
    float med1, med2, density;
    int have;        // number of medians recorded (0, 1, 2+)
    bool active;     // a window pass is under way this iteration
    float lo, hi;    // the window
    uint32_t below;  // per wave: distances below lo
    uint32_t kept;   // per wave: distances kept (kOverflow once the region is full)
    uint32_t wshift; // window histogram bin of a kept distance: (key - key(lo)) >> wshift
    uint32_t *whist; // its 256 counters (zero before the walk)
    int wcap;        // per-wave capacity of the window buffer

    __device__ void reset(int cap = kWinRegion)
    {
        med1 = med2 = density = 0.f;
        have = 0;
        active = false;
        wcap = cap;
    }

    // window of this iteration (active only with a previous median)
    __device__ void plan(uint32_t *hist256)
    {
        whist = hist256;
        active = have >= 1 && med1 > 0.f;
        below = 0;
        kept = 0;
        if (!active) return;
        const float move = have >= 2 ? fabsf(med1 - med2) : 0.f;
        const float pred = have >= 2 ? med1 + (med1 - med2) : med1;
        float w = density > 0.f ? (float)kWinTarget / (2.f * density) : 1e-3f * med1;
        w = fmax_(w, 3.f * move);
        w = fmax_(w, 2e-5f * med1);
        lo = uniform(fmax_(pred - w, 0.f));
        hi = uniform(pred + w);
        const uint32_t span = __float_as_uint(hi) - __float_as_uint(lo);
        const int bits = span == 0 ? 1 : 32 - __clz(span);
        wshift = bits > 8 ? bits - 8 : 0;
    }

    static constexpr uint32_t kOverflow = 0x40000000u;

    // One tile of distances (diag: only pairs k > i count).  The common case
    // is two comparisons per distance, D < lo and D < hi, as wave masks: the
    // wave's count below lo is the population count of the first (scalar
    // work), and D lies in the window [lo, hi) where the second holds and the
    // first does not (a NaN is in neither; -0 counts as 0).  Only a tile
    // holding window distances appends them to the wave's region, binned by
    // key(D) - key(lo) on the bit patterns.
    __device__ void visit(f32x4 Dv, bool diag, float *region)
    {
        if (diag) {
            const int l = threadIdx.x & 63;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (!((diag_lanes(r) >> l) & 1ull)) Dv[r] = __builtin_huge_valf();
        }
        unsigned long long win[4], any = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const unsigned long long mlo = __builtin_amdgcn_ballot_w64(Dv[r] < lo);
            const unsigned long long mhi = __builtin_amdgcn_ballot_w64(Dv[r] < hi);
            below += (uint32_t)__builtin_popcountll(mlo);
            win[r] = mhi & ~mlo;
            any |= win[r];
        }
        if (any) {
            const uint32_t klo = __float_as_uint(lo);
            const int l = threadIdx.x & 63;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const unsigned long long mk = win[r];
                const uint32_t cnt = (uint32_t)__builtin_popcountll(mk);
                const bool fits = kept + cnt <= (uint32_t)wcap;  // kOverflow stays
                if (fits && ((mk >> l) & 1ull)) {
                    const float v = Dv[r] + 0.f;  // no -0
                    region[kept + lanes_below(mk)] = v;
                    atomicAdd(&whist[(__float_as_uint(v) - klo) >> wshift], 1u);
                }
                kept = fits ? kept + cnt : kOverflow;
            }
        }
    }

    // After every wave has visited its tiles (no barrier needed before the
    // call).  Returns the exact lower median.
    template <bool K4>
    __device__ float finish(const float *X8, int n, int npad, float *buf, uint32_t *hist, uint32_t *red)
    {
        const uint32_t M = (uint32_t)((long)n * (n - 1) / 2);
        if (M == 0) return __builtin_nanf("");
        const uint32_t rank = (M - 1) / 2;
        const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = wave_id(), nwaves = nt >> 6;
        // red[0..1] radix selection, red[2..6] window_select, red[8..9]
        // buffer_select
        uint32_t *wcnt = red + 10;    // per-wave kept counts (red[10..25])
        uint32_t *wbelow = red + 26;  // per-wave below counts (red[26..41])
        float med = 0.f;
        bool done = false;
        if (active) {
            if (lane == 0) {
                wbelow[wave] = below;
                wcnt[wave] = kept;
            }
            __syncthreads();
            uint32_t cnt_lo = 0, n_in = 0;
            bool overflow = false;
            for (int q = 0; q < nwaves; ++q) {
                cnt_lo += wbelow[q];
                n_in += wcnt[q];
                overflow |= wcnt[q] > (uint32_t)wcap;
            }
            density = uniform((float)n_in / (hi - lo));
            if (!overflow && rank >= cnt_lo && rank < cnt_lo + n_in) {
                med = window_select(buf, wcnt, nwaves, wcap, rank - cnt_lo, __float_as_uint(lo), __float_as_uint(hi),
                                    wshift, whist, red, (float *)whist);
                done = true;
            }
            __syncthreads();
        }
        if (!done) med = radix_median_mfma<K4>(X8, npad, rank, hist, red);
        med = uniform(med);
        med2 = med1;
        med1 = med;
        have = have < 2 ? have + 1 : 2;
        active = false;
        return med;
    }
};

// Wave priority from progress relative to the waves that share the SIMD
// (waves w, w + 4, w + 8, w + 12 of a workgroup).  The SIMD arbiter serves
// the oldest wave first among equal priorities, so without this a pass ends
// in age order and its tail runs on one or two waves, too few to hide
// latency.  Every second tile step a wave publishes its running count of
// steps in LDS and reads its mates' counts; the read is only used at the
// next call, so it never waits.  A wave ahead of its slowest mate yields:
// priority 3 within 2 steps of it, 2 within 4, 1 within 8, else 0.
struct ProgressBalance {
    typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
    // the words are addressed as LDS (ds instructions, no vector-memory wait)
    typedef __attribute__((address_space(3))) volatile uint32_t lds_u32;
    typedef __attribute__((address_space(3))) volatile u32x4_t lds_u32x4;
    lds_u32x4 *row;       // the SIMD's four counts
    lds_u32 *own;         // this wave's count
    uint32_t done;        // steps of this wave so far (all passes)
    uint32_t mn;          // the least of the four counts at the last step

    // prog: 16 LDS words set to ~0 (absent waves never lag) before a barrier
    __device__ void init(uint32_t *prog, int wave)
    {
        row = (lds_u32x4 *)(prog + (wave & 3) * 4);
        own = (lds_u32 *)(prog + (wave & 3) * 4 + (wave >> 2));
        done = 0;
        mn = 0;
    }
    __device__ void step()
    {
        done += 2;
        const uint32_t ahead = done - min(mn, done);
        if (ahead <= 2) __builtin_amdgcn_s_setprio(3);
        else if (ahead <= 4) __builtin_amdgcn_s_setprio(2);
        else if (ahead <= 8) __builtin_amdgcn_s_setprio(1);
        else __builtin_amdgcn_s_setprio(0);
        *own = done;
        const u32x4_t p = *row;
        mn = __builtin_amdgcn_readfirstlane(min(min(p[0], p[1]), min(p[2], p[3])));
    }
};

// One sequence's time step (b: its index in the strided batch of `a`).  The
// workgroup owns the sequence: all state in LDS, every barrier block-wide.
// Sum of a value over the four 16-lane rows of a wave, in every lane.
__device__ __forceinline__ float sum_row_quarters(float v)
{
    auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(s[0]) + __uint_as_float(s[1]);
    s = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}

// Given four values v0..v3 of a wave, lane l in 16-lane row w receives the
// sum of v_w over the four rows, in that lane's column (a transpose of rows
// against values, then a sum): two rounds of lane swaps.
__device__ __forceinline__ float sum_quarters_scatter(float v0, float v1, float v2, float v3)
{
    auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(v0), __float_as_uint(v2), false, false);
    auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(v1), __float_as_uint(v3), false, false);
    // lanes 0..31: v0 (resp. v1) over rows r, r + 2; lanes 32..63: v2 (v3)
    const float s0 = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    const float s1 = __uint_as_float(b[0]) + __uint_as_float(b[1]);
    auto c = __builtin_amdgcn_permlane16_swap(__float_as_uint(s0), __float_as_uint(s1), false, false);
    return __uint_as_float(c[0]) + __uint_as_float(c[1]);
}

// ---- multi-workgroup mode ---------------------------------------------
// The G workgroups of one sequence each own tasks_local = ntasks / G
// consecutive 64-particle target tasks and hold every particle in LDS.  Per
// SVGD iteration they exchange, through global memory, the score rows of
// their targets and their share of the median's window pass (barrier 1),
// then their moved particles (barrier 2); every workgroup then holds the
// same state, and every selection they make from the exchanged data (the
// median, the radix fallback) is the same.  The layout of one sequence's
// exchange area, host and device:
constexpr int kCoopWinCap = 2048;     // window buffer of a workgroup (floats)
constexpr uint32_t kCoopSpinLimit = 1u << 24;  // barrier wait bound (polls)

struct CoopLayout {
    long off_ctr, off_x, off_s, off_info, off_whist, off_vals, off_rhist, bytes;
    __host__ __device__ CoopLayout(int npad, int G)
    {
        long o = 0;
        off_ctr = o; o += 256;
        off_x = o; o += align16((long)npad * 8 * 4);
        off_s = o; o += align16((long)npad * 8 * 4);
        off_info = o; o += align16((long)G * 4 * 4);
        off_whist = o; o += align16((long)G * 256 * 4);
        off_vals = o; o += align16((long)G * kCoopWinCap * 4);
        off_rhist = o; o += align16((long)2 * G * kBins * 4);   // two buffers, alternate passes
        bytes = (o + 255) / 256 * 256;
    }
};

struct CoopArgs {
    char *base;     // exchange area of sequence 0; sequence b at base + b * stride
    long stride;
    int G;          // workgroups per sequence
    int gi;         // this workgroup's index within its sequence (set by the kernel)
};

// Barrier among the G workgroups of a sequence: thread 0 makes the
// workgroup's global writes visible at device scope, arrives on the counter
// and waits for epoch * G arrivals (bounded: past the bound the stall bit is
// set and the wait ends, and once it is set no barrier of the run waits),
// then acquires before the workgroup reads what the others wrote.
__device__ __forceinline__ void coop_barrier(uint32_t *ctr, uint32_t target, uint32_t *status)
{
    // every wave waits for its own global stores to complete, so they sit in
    // the L2 before the workgroup barrier; thread 0's device-scope release
    // then writes them back, and its acquire (before the second workgroup
    // barrier) invalidates the caches the other waves read through: one
    // write-back and one invalidation per workgroup
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(ctr, 1u);
        uint32_t polls = 0;
        // after one stall no later barrier waits (the run is flagged already)
        const bool stalled = (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & STATUS_STALLED) != 0;
        while (!stalled && __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++polls > kCoopSpinLimit) {
                atomicOr(status, STATUS_STALLED);
                break;
            }
        }
        __threadfence();
    }
    __syncthreads();
}

// SPLIT: the layout splits the sources of each task among waves (MfmaLds
// ns_max > 1); a separate instantiation, so the unsplit path keeps its
// registers.  COOP (with SPLIT): one of the G workgroups of sequence b in
// the multi-workgroup mode (cx).
template <int KIND, int D, int TS, bool SPLIT, bool COOP = false>
__device__ __forceinline__ void step_mfma_body(const StepArgs<float> &a, const int b, const CoopArgs cx = CoopArgs{})
{
    using F = Family<float, KIND, D>;
    using R = RealOps<float>;
    static_assert(D <= 7, "K-column 7 carries the norms");
    extern __shared__ __align__(16) unsigned char smem[];
    static_assert(!COOP || SPLIT, "the multi-workgroup mode splits the sources");
    // d <= 3: four K-rows per tile (coordinates and the norm or constant in
    // row 3) and four rows of sums, one MFMA each where d <= 7 takes two
    constexpr bool K4 = D <= 3;
    const int n = a.n, np = a.n_prev;
    const int G = COOP ? cx.G : 1, gi = COOP ? cx.gi : 0;
    const int npad0 = (n + 63) / 64 * 64;
    const MfmaLds L(n, np, (int)(blockDim.x >> 6), COOP ? npad0 / 64 / G : 0, COOP ? kCoopWinCap : kWinCap);
    const int npad = L.npad, nppad = L.nppad;
    constexpr bool split = SPLIT;               // sources of a task split among waves (L.ns_max > 1)
    float *PART = (float *)(smem + L.off_part); // [ns_max][ntasks * 64][kPartStride] partial sums of the splits
    // the workgroup's targets: tasks [tbase / 64, tbase / 64 + ntasks) (all of them outside COOP)
    const int tbase = gi * L.ntasks * 64;
    // exchange area of this sequence (COOP)
    const CoopLayout CL(npad, G);
    char *cbase = COOP ? cx.base + (long)b * cx.stride : nullptr;
    uint32_t *cctr = (uint32_t *)(cbase + CL.off_ctr);
    float *cX = (float *)(cbase + CL.off_x);
    float *cS = (float *)(cbase + CL.off_s);
    uint32_t *cinfo = (uint32_t *)(cbase + CL.off_info);
    uint32_t *cwhist = (uint32_t *)(cbase + CL.off_whist);
    float *cvals = (float *)(cbase + CL.off_vals);
    uint32_t *crhist = (uint32_t *)(cbase + CL.off_rhist);
    uint32_t epoch = 0;  // barriers passed (the same count in every workgroup)
    float *X8 = (float *)(smem + L.off_x);     // [npad][8]  centred particles, |x|^2 in column 7 (pad: 0.., +inf)
    float *S8 = (float *)(smem + L.off_s);     // [npad][8]  scores
    float *VT = (float *)(smem + L.off_m);     // [9][nppad] rows 2 mh_c (c < 7; 0 for c >= d), 1, c'_j
    float *PHP = (float *)(smem + L.off_phip); // [nppad] previous forward-recursion scores
    uint32_t *hist = (uint32_t *)(smem + L.off_scr);
    float *WIN = (float *)(smem + L.off_win);                    // median window buffer
    uint32_t *whist = (uint32_t *)(smem + L.off_win) + L.win_cap;  // its histogram
    float *sz = (float *)(smem + L.off_z);
    uint8_t *smask = smem + L.off_mask;
    uint32_t *red = (uint32_t *)(smem + L.off_red);
    float *redf = (float *)(smem + L.off_red + 256);

    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = wave_id(), nwaves = nt >> 6;
    const int g = lane >> 4, col = lane & 15;
    const DevModel<float> &m = a.m;
    const float *xprev = a.x_prev + (long)b * a.x_prev_stride;
    float *xg = a.x + (long)b * a.x_stride;
    const float inf = R::inf();

    for (int o = tid; o < 16; o += nt) red[kProgSlot + o] = 0xffffffffu;
    // wave priorities by progress: with whole tasks per wave (the arm7
    // shape: 64 tile steps per pass) the balancing pays (5%), and in the
    // multi-workgroup step (2% at arm7 B = 1); one workgroup with sources
    // split among waves runs short passes where it costs more than it saves
    // (range2d 5%), so that kernel leaves it out
    ProgressBalance bal;
    bal.init(red + kProgSlot, wave);
    constexpr bool kBalance = !SPLIT || COOP;
    for (int o = tid; o < m.obs_dim; o += nt) sz[o] = a.z[(long)b * a.z_stride + o];
    const uint8_t *mk = nullptr;
    if (a.mask) {
        for (int o = tid; o < m.n_obs; o += nt) smask[o] = a.mask[(long)b * a.mask_stride + o];
        mk = smask;
    }
    float rs[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) rs[c] = c < D ? m.rs[c] : 0.f;

    // reference point: mean of the transition means
    float ref[D];
    for (int c = 0; c < D; ++c) {
        float part = 0.f;
        for (int j = tid; j < np; j += nt) {
            float xp[D], mu[D];
#pragma unroll
            for (int q = 0; q < D; ++q) xp[q] = xprev[(long)j * D + q];
            F::mean(m, a.t, xp, mu);
            part += mu[c];
        }
        part = wave_sum(part);
        if (lane == 0) redf[wave] = part;
        __syncthreads();
        float tot = 0.f;
        for (int w = 0; w < nwaves; ++w) tot += redf[w];
        ref[c] = uniform(tot / (float)np);
        __syncthreads();
    }

    // transition means, centred and log2-scaled, component-major:
    // VT[c][j] = 2 mh_jc (c < 7), VT[7][j] = 1, VT[8][j] = c'_j =
    // log2 w_j - |mh_j|^2; pad columns give logit -inf
    for (int j = tid; j < nppad; j += nt) {
        float row[kVtRows];
#pragma unroll
        for (int c = 0; c < kVtRows; ++c) row[c] = 0.f;
        row[7] = 1.f;
        if (j < np) {
            float xp[D], mu[D];
#pragma unroll
            for (int q = 0; q < D; ++q) xp[q] = xprev[(long)j * D + q];
            F::mean(m, a.t, xp, mu);
            float nrm = 0.f;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const float mh = (mu[c] - ref[c]) * rs[c];
                row[c] = 2.f * mh;
                nrm += mh * mh;
            }
            const float lw = a.log_w ? a.log_w[(long)b * a.log_w_stride + j] : -R::log_((float)np);
            row[8] = lw * (float)kLog2e - nrm;
        } else {
            row[8] = -inf;
        }
#pragma unroll
        for (int c = 0; c < kVtRows; ++c) VT[(long)c * nppad + j] = row[c];
    }
    // initial particles, centred
    for (int i = tid; i < npad; i += nt) {
        float xi[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) xi[c] = 0.f;
        if (i < n) {
            if (a.init_given) {
#pragma unroll
                for (int c = 0; c < D; ++c) xi[c] = xg[(long)i * D + c] - ref[c];
            } else {
                float xp[D], mu[D];
                const int j = i % np;
#pragma unroll
                for (int c = 0; c < D; ++c) xp[c] = xprev[(long)j * D + c];
                F::mean(m, a.t, xp, mu);
                double nz[D];
                normals<D>(a.seed, a.seq_offset + (uint32_t)b, (uint32_t)a.t, (uint32_t)i, nz);
#pragma unroll
                for (int c = 0; c < D; ++c) xi[c] = (mu[c] + m.sqrt_q[c] * (float)nz[c]) - ref[c];
            }
        }
        float nrm = 0.f;
#pragma unroll
        for (int c = 0; c < 7; ++c) nrm += xi[c] * xi[c];
        xi[7] = i < n ? nrm : inf;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            X8[(long)i * 8 + c] = xi[c];
            S8[(long)i * 8 + c] = 0.f;
        }
    }
    __syncthreads();

    // mean of the centred transition means (literal score reading)
    float mbar_all[D];
#pragma unroll
    for (int c = 0; c < D; ++c) mbar_all[c] = 0.f;
    if (a.do_svgd && a.trans_mode == 1) {
        for (int c = 0; c < D; ++c) {
            float part = 0.f;
            for (int j = tid; j < np; j += nt) part += VT[(long)c * nppad + j] * 0.5f / rs[c];
            part = wave_sum(part);
            if (lane == 0) redf[wave] = part;
            __syncthreads();
            float tot = 0.f;
            for (int w = 0; w < nwaves; ++w) tot += redf[w];
            mbar_all[c] = uniform(tot / (float)np);
            __syncthreads();
        }
    }

    const int ntasks = L.ntasks;   // target tasks of this workgroup
    const int njt = nppad / 16;
    // every workgroup of the sequence has read its inputs before any writes
    // its outputs (the x array may hold the initial particles)
    if (COOP) coop_barrier(cctr, ++epoch * (uint32_t)G, a.status);
    const int nkt = npad / 16;
    const float inv_n = 1.f / (float)n;
    float h = 1.f;
    MedianTracker tracker;
    tracker.reset(L.win_region);

    for (int it = 0; a.do_svgd && it < a.n_iter; ++it) {
        // (1) the bandwidth needs the exact lower median of the squared
        // distances of the current particles; its window pass is spread over
        // the score pass, which leaves the particles unchanged
        const bool need_median = a.bw_mode == 0 || it == 0;
        if (need_median) tracker.plan(whist);
        TileWalker<K4, COOP> walker;
        if (tracker.active) {
            if (COOP)
                walker.start(X8, npad, g, col, gi * nwaves + wave, G * nwaves);
            else
                walker.start(X8, npad, g, col);
        }
        float *wregion = WIN + wave * L.win_region;
        auto walk_step = [&]() {
            f32x4 W0, W1;
            walker.issue(X8, g, col, W0, W1);
            tracker.visit(W0, false, wregion);
            if (walker.second()) tracker.visit(W1, false, wregion);
            walker.advance(X8, g, col);
        };

        // (2) scores
        // score_sums: osum = sum_j e_kj [2 mh_j, 1] over the source tiles
        // [j0, j1) for this lane's particle kbase + lane, relative to the
        // reference sref (e_kj = exp2(logit_kj - sref))
        auto score_sums = [&](int kbase, int j0, int j1, float (&osum)[8], float &sref) {
            {
                f32x4 cm[kTilesPerWave];  // -reference of each particle column, as the accumulator input
                float bx0[kTilesPerWave], bx1[kTilesPerWave];
#pragma unroll
                for (int q = 0; q < kTilesPerWave; ++q) {
                    const int kk = kbase + 16 * q + col;
                    const int kd0 = g, kd1 = 4 + g;
                    bx0[q] = kd0 < D ? X8[(long)kk * 8 + kd0] * rs[kd0] : (K4 && kd0 == 3 ? 1.f : 0.f);
                    bx1[q] = kd1 < D ? X8[(long)kk * 8 + kd1] * rs[kd1] : (kd1 == 7 ? 1.f : 0.f);
                    cm[q] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
                // Sums on the 4x4x1 (16-block) MFMA straight from the logit
                // tile layout: register r of lane l holds e of source
                // 16 jt + 4 (l / 16) + r and particle kbase + 16 q + l % 16, so
                // block b = l / 4 takes B = that register and A = table rows
                // 4 ch + l % 4 of its source; lane l of O4[ch][q] accumulates
                // rows 4 ch + i (register i) of particle kbase + 16 q + l % 16
                // over the source quarter l / 16.  With K4 one group holds
                // rows 2 mh_0..2 and the 1 (table row 7) as its row 3.
                constexpr int NGS = K4 ? 1 : 2;
                f32x4 O4[NGS][kTilesPerWave];
#pragma unroll
                for (int ch = 0; ch < NGS; ++ch)
#pragma unroll
                    for (int q = 0; q < kTilesPerWave; ++q) O4[ch][q] = f32x4{0.f, 0.f, 0.f, 0.f};
                // four consecutive sources 4 (l / 16) + r of rows l % 4, 4 + l % 4
                const float *vt0 = VT + (long)(K4 && (lane & 3) == 3 ? 7 : (lane & 3)) * nppad + 4 * g;
                const float *vt1 = VT + (long)(4 + (lane & 3)) * nppad + 4 * g;
                // logit A operands: K-row g (2 mh), K-row 4 + g (row 7 of the
                // table, the 1, becomes c'_j in K-row 7); with K4, c'_j in
                // K-row 3 of the one chunk
                const float *am0p = VT + (long)(K4 && g == 3 ? 8 : g) * nppad + col;
                const float *am1p = VT + (long)(g == 3 ? 8 : 4 + g) * nppad + col;
                // logits of tile jt relative to the column references
                auto logits = [&](int jt, f32x4 (&Lo)[kTilesPerWave]) {
                    const float am0 = am0p[jt * 16];
#pragma unroll
                    for (int q = 0; q < kTilesPerWave; ++q) Lo[q] = mfma16(am0, bx0[q], cm[q]);
                    if (!K4) {
                        const float am1 = am1p[jt * 16];
#pragma unroll
                        for (int q = 0; q < kTilesPerWave; ++q) Lo[q] = mfma16(am1, bx1[q], Lo[q]);
                    }
                };
                // Raises the reference of the columns of a relative logit tile
                // whose maximum lies more than 2^64 above it (all four lane
                // groups of a column agree), rescaling the sums and the tile;
                // with `first`, sets the references to the tile's maxima.  The
                // test compares the bit patterns as integers: for a positive
                // bound that orders like the floats, and NaN also triggers.
                auto rebase = [&](f32x4 (&T)[kTilesPerWave], bool first) {
                    int mxi = __float_as_int(T[0][0]);
#pragma unroll
                    for (int q = 0; q < kTilesPerWave; ++q)
#pragma unroll
                        for (int r = 0; r < 4; ++r) mxi = max(mxi, __float_as_int(T[q][r]));
                    if (first || __builtin_amdgcn_ballot_w64(mxi > __float_as_int(kRescaleGap))) {
                        float shq[kTilesPerWave];
#pragma unroll
                        for (int q = 0; q < kTilesPerWave; ++q) {
                            const float lmax = fmax_(fmax_(T[q][0], T[q][1]), fmax_(T[q][2], T[q][3]));
                            const float gm = group_max4(lmax);
                            const bool up = first ? gm > -inf : gm > kRescaleGap;
                            shq[q] = up ? gm : 0.f;
                            T[q] -= shq[q];
                            cm[q] -= shq[q];
                        }
                        if (!first) {
#pragma unroll
                            for (int q = 0; q < kTilesPerWave; ++q) {
                                const float sc = R::exp2_(-shq[q]);
#pragma unroll
                                for (int ch = 0; ch < NGS; ++ch) O4[ch][q] *= sc;
                            }
                        }
                    }
                };
                // One logit tile per step; with WALK, two tiles of the median
                // window pass ride along.
                auto score_loop = [&](auto walk_tag) {
                    constexpr bool WALK = decltype(walk_tag)::value;
                    // exponentials and sums of a relative logit tile; with
                    // WALK the median walk's two tiles W0, W1 (issued before
                    // the logits are checked) are visited after the sums
                    auto body = [&](int jt, f32x4 (&T)[kTilesPerWave], const f32x4 &W0, const f32x4 &W1) {
                        f32x4 va[NGS];
                        va[0] = *(const f32x4 *)(vt0 + jt * 16);
                        if (!K4) va[NGS - 1] = *(const f32x4 *)(vt1 + jt * 16);
#pragma unroll
                        for (int q = 0; q < kTilesPerWave; ++q)
#pragma unroll
                            for (int r = 0; r < 4; ++r) T[q][r] = R::exp2_(T[q][r]);
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int q = 0; q < kTilesPerWave; ++q)
#pragma unroll
                                for (int ch = 0; ch < NGS; ++ch)
                                    O4[ch][q] = __builtin_amdgcn_mfma_f32_4x4x1f32(va[ch][r], T[q][r], O4[ch][q], 0,
                                                                                   0, 0);
                        if (WALK && !walker.done()) {
                            tracker.visit(W0, false, wregion);
                            if (walker.second()) tracker.visit(W1, false, wregion);
                            walker.advance(X8, g, col);
                        }
                    };
                    if (WALK) {
                        // one buffer (the walk's registers leave no room for
                        // two); the walk's MFMAs go between the logits and
                        // their check, which waits for them
                        f32x4 T[kTilesPerWave], W0, W1;
                        logits(j0, T);
                        walker.issue(X8, g, col, W0, W1);
                        rebase(T, true);
                        body(j0, T, W0, W1);
                        for (int jt = j0 + 1; jt < j1; ++jt) {
                            if (kBalance && (jt & 1) == 0) bal.step();
                            logits(jt, T);
                            walker.issue(X8, g, col, W0, W1);
                            rebase(T, false);
                            body(jt, T, W0, W1);
                        }
                    } else {
                        // the logits of tile jt + 1 are issued (and checked)
                        // around the exponentials and sums of tile jt
                        const f32x4 none = {0.f, 0.f, 0.f, 0.f};
                        auto tile = [&](int jt, f32x4 (&T)[kTilesPerWave], f32x4 (&Tn)[kTilesPerWave]) {
                            logits(min(jt + 1, j1 - 1), Tn);
                            body(jt, T, none, none);
                            rebase(Tn, false);
                        };
                        f32x4 TA[kTilesPerWave], TB[kTilesPerWave];
                        logits(j0, TA);
                        rebase(TA, true);
                        for (int jt = j0; jt < j1; jt += 2) {
                            if (kBalance) bal.step();
                            tile(jt, TA, TB);
                            if (jt + 1 < j1) tile(jt + 1, TB, TA);
                        }
                    }
                };
                if (tracker.active && !walker.done())
                    score_loop(std::true_type{});
                else
                    score_loop(std::false_type{});
                // lane l takes particle kbase + l: tile q = l / 16, summed
                // over the four source quarters; its reference is the one of
                // column l % 16 of tile q, which lane l holds
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    osum[i] = sum_quarters_scatter(O4[0][0][i], O4[0][1][i], O4[0][2][i], O4[0][3][i]);
                    if (!K4)
                        osum[4 + i] = sum_quarters_scatter(O4[NGS - 1][0][i], O4[NGS - 1][1][i], O4[NGS - 1][2][i],
                                                           O4[NGS - 1][3][i]);
                }
                if (K4) {
                    // the sum of e sits in row 3; rows 3..6 carry nothing
                    osum[7] = osum[3];
#pragma unroll
                    for (int i = 3; i < 7; ++i) osum[i] = 0.f;
                }
                const int qq = lane >> 4;
                float cref = cm[0][0];
#pragma unroll
                for (int q = 1; q < kTilesPerWave; ++q) cref = qq == q ? cm[q][0] : cref;
                sref = -cref;
            }
        };
        if (split) {
            // this wave's split of its task's sources: partial sums to LDS,
            // merged per particle once h is known
            if (a.trans_mode == 0 && wave < ntasks * L.ns_sc) {
                const int task = wave % ntasks, sp = wave / ntasks;
                float osum[8], sref;
                score_sums(tbase + task * 64, sp * njt / L.ns_sc, (sp + 1) * njt / L.ns_sc, osum, sref);
                float *pp = PART + ((long)sp * ntasks * 64 + task * 64 + lane) * kPartStride;
#pragma unroll
                for (int c = 0; c < 8; ++c) pp[c] = osum[c];
                pp[8] = sref;
            }
        }
        for (int task = wave; !split && task < ntasks; task += nwaves) {
            const int kbase = task * 64;
            float osum[8];  // trans_mode 0: sum_j e_kj [2 mh_j, 1] of this lane's particle kbase + lane
            if (a.trans_mode == 0) {
                float sref;
                score_sums(kbase, 0, njt, osum, sref);
            }
            {
                const int k = kbase + lane;
                float srow[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) srow[c] = 0.f;
                srow[7] = 1.f;  // the Stein pass sums kappa through this column
                if (k < n) {
                    float xt[D], xa[D], gr[D];
#pragma unroll
                    for (int c = 0; c < D; ++c) {
                        xt[c] = X8[(long)k * 8 + c];
                        xa[c] = xt[c] + ref[c];
                    }
                    F::grad(m, sz, mk, xa, gr);
                    if (a.trans_mode == 0) {
                        const float inv_sum = 1.f / osum[7];
#pragma unroll
                        for (int c = 0; c < D; ++c) {
                            const float mb = osum[c] * inv_sum * 0.5f / rs[c];
                            srow[c] = gr[c] - (xt[c] - mb) * m.inv_q[c];
                        }
                    } else {
#pragma unroll
                        for (int c = 0; c < D; ++c) srow[c] = gr[c] - (xt[c] - mbar_all[c]) * m.inv_q[c];
                    }
                }
#pragma unroll
                for (int c = 0; c < 8; ++c) S8[(long)k * 8 + c] = srow[c];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        __builtin_amdgcn_s_setprio(0);
        if (tracker.active) {
            while (!walker.done()) walk_step();
            walker.diagonals(X8, g, col, [&](const f32x4 &Dd, bool dg) { tracker.visit(Dd, dg, wregion); });
        }
        __syncthreads();
        if constexpr (COOP) {
            // score rows of this workgroup's targets from the splits' partial
            // sums (rebased to their largest reference, summed in split
            // order), to the exchange area: the largest reference per target,
            // the rebased sums per (target, row) into S8, then the rows
            const int ntl = ntasks * 64;
            float *mref = (float *)hist;  // [ntl] (the radix histogram is free here)
            if (a.trans_mode == 0) {
                for (int kl = tid; kl < ntl; kl += nt) {
                    float mx = -inf;
                    for (int sp = 0; sp < L.ns_sc; ++sp)
                        mx = fmax_(mx, PART[((long)sp * ntl + kl) * kPartStride + 8]);
                    mref[kl] = mx;
                }
                __syncthreads();
                for (int e = tid; e < ntl * 8; e += nt) {
                    const int kl = e >> 3, c = e & 7;
                    const float mx = mref[kl];
                    float acc = 0.f;
                    for (int sp = 0; sp < L.ns_sc; ++sp) {
                        const float *pp = PART + ((long)sp * ntl + kl) * kPartStride;
                        acc += pp[c] * R::exp2_(pp[8] - mx);
                    }
                    S8[(long)(tbase + kl) * 8 + c] = acc;
                }
                __syncthreads();
            }
            for (int kl = tid; kl < ntl; kl += nt) {
                const int k = tbase + kl;
                float srow[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) srow[c] = 0.f;
                srow[7] = 1.f;
                if (k < n) {
                    float xt[D], xa[D], gr[D];
#pragma unroll
                    for (int c = 0; c < D; ++c) {
                        xt[c] = X8[(long)k * 8 + c];
                        xa[c] = xt[c] + ref[c];
                    }
                    F::grad(m, sz, mk, xa, gr);
                    if (a.trans_mode == 0) {
                        const float inv_sum = 1.f / S8[(long)k * 8 + 7];
#pragma unroll
                        for (int c = 0; c < D; ++c) {
                            const float mb = S8[(long)k * 8 + c] * inv_sum * 0.5f / rs[c];
                            srow[c] = gr[c] - (xt[c] - mb) * m.inv_q[c];
                        }
                    } else {
#pragma unroll
                        for (int c = 0; c < D; ++c) srow[c] = gr[c] - (xt[c] - mbar_all[c]) * m.inv_q[c];
                    }
                }
#pragma unroll
                for (int c = 0; c < 8; ++c) cS[(long)k * 8 + c] = srow[c];
            }
            // this workgroup's share of the window pass: counts, its kept
            // distances in wave order, its histogram
            if (need_median && tracker.active) {
                if (lane == 0) {
                    red[26 + wave] = tracker.below;
                    red[10 + wave] = tracker.kept;
                }
                __syncthreads();
                uint32_t below = 0, kept = 0, off_w = 0;
                bool ovf = false;
                for (int q = 0; q < nwaves; ++q) {
                    const uint32_t c = red[10 + q];
                    ovf |= c > (uint32_t)L.win_region;
                    if (q < wave) off_w += c;
                    below += red[26 + q];
                    kept += c;
                }
                if (!ovf)
                    for (uint32_t q = lane; q < tracker.kept; q += kWave)
                        cvals[(long)gi * kCoopWinCap + off_w + q] = wregion[q];
                for (int q = tid; q < 256; q += nt) cwhist[gi * 256 + q] = whist[q];
                if (tid == 0) {
                    cinfo[gi * 4 + 0] = below;
                    cinfo[gi * 4 + 1] = ovf ? 0u : kept;
                    cinfo[gi * 4 + 2] = ovf ? 1u : 0u;
                }
            }
            coop_barrier(cctr, ++epoch * (uint32_t)G, a.status);
            // every score row
            for (int k = tid; k < npad; k += nt)
#pragma unroll
                for (int c = 0; c < 8; ++c) S8[(long)k * 8 + c] = cS[(long)k * 8 + c];
            if (need_median) {
                // the median from every workgroup's share: the same value in all
                const uint32_t M = (uint32_t)((long)n * (n - 1) / 2);
                const uint32_t rank = M > 0 ? (M - 1) / 2 : 0u;
                float med = __builtin_nanf("");
                bool done = M == 0;
                if (!done && tracker.active) {
                    // the workgroups' counts, staged in LDS (one global round trip)
                    uint32_t *ci = (uint32_t *)redf;  // [16] kept, [16] below, [16] overflow
                    if (tid < G) {
                        ci[tid] = cinfo[tid * 4 + 1];
                        ci[16 + tid] = cinfo[tid * 4 + 0];
                        ci[32 + tid] = cinfo[tid * 4 + 2];
                    }
                    __syncthreads();
                    uint32_t below = 0, nin = 0;
                    bool ovf = false;
                    for (int q = 0; q < G; ++q) {
                        below += ci[16 + q];
                        nin += ci[q];
                        ovf |= ci[32 + q] != 0u;
                    }
                    tracker.density = uniform((float)nin / (tracker.hi - tracker.lo));
                    if (!ovf && rank >= below && rank < below + nin && nin <= (uint32_t)L.win_cap) {
                        // every workgroup's kept distances into this one's window
                        // buffer (workgroup order), their histogram, then the
                        // window selection of the one-workgroup kernel
                        for (uint32_t e = tid; e < nin; e += nt) {
                            uint32_t off = 0;
                            int gg = 0;
                            while (e >= off + ci[gg]) {
                                off += ci[gg];
                                ++gg;
                            }
                            WIN[e] = cvals[(long)gg * kCoopWinCap + (e - off)];
                        }
                        for (int q = tid; q < 256; q += nt) whist[q] = 0;
                        if (tid == 0) red[10] = nin;
                        __syncthreads();
                        const uint32_t klo = __float_as_uint(tracker.lo);
                        for (uint32_t e = tid; e < nin; e += nt)
                            atomicAdd(&whist[(__float_as_uint(WIN[e]) - klo) >> tracker.wshift], 1u);
                        __syncthreads();
                        med = window_select(WIN, red + 10, 1, L.win_cap, rank - below, klo,
                                            __float_as_uint(tracker.hi), tracker.wshift, whist, red, (float *)whist);
                        done = true;
                    } else if (!ovf && rank >= below && rank < below + nin) {
                        // more kept distances than this buffer holds: the summed
                        // histograms locate the median's bin, and only that bin's
                        // distances are gathered
                        const uint32_t r = rank - below;
                        for (int q = tid; q < 256; q += nt) {
                            uint32_t c = 0;
                            for (int gg = 0; gg < G; ++gg) c += cwhist[gg * 256 + q];
                            whist[q] = c;
                        }
                        __syncthreads();
                        if (wave == 0) {
                            typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
                            const u32x4_t c = *(const u32x4_t *)(whist + lane * 4);
                            const uint32_t cnt = c[0] + c[1] + c[2] + c[3];
                            const uint32_t incl = wave_incl_scan(cnt, lane);
                            const uint32_t excl = incl - cnt;
                            if (r >= excl && r < incl) {
                                uint32_t rr = r - excl;
#pragma unroll
                                for (int q = 0; q < 4; ++q) {
                                    if (rr < c[q]) {
                                        red[2] = (uint32_t)(lane * 4 + q);
                                        red[3] = rr;
                                        red[4] = c[q];
                                        break;
                                    }
                                    rr -= c[q];
                                }
                            }
                            if (lane == 0) red[6] = 0;
                        }
                        __syncthreads();
                        const uint32_t bin = red[2], rr = red[3], cb = red[4];
                        if (cb <= (uint32_t)kWave) {
                            float *cand = (float *)whist;  // the histogram is dead once the bin is known
                            const uint32_t klo = __float_as_uint(tracker.lo);
                            for (int gg = 0; gg < G; ++gg) {
                                const uint32_t cnt = ci[gg];
                                for (uint32_t q = tid; q < cnt; q += nt) {
                                    const float v = cvals[(long)gg * kCoopWinCap + q];
                                    if (((__float_as_uint(v) - klo) >> tracker.wshift) == bin)
                                        cand[atomicAdd(&red[6], 1u)] = v;
                                }
                            }
                            __syncthreads();
                            if (wave == 0 && (uint32_t)lane < cb) {
                                const float v = cand[lane];
                                uint32_t less = 0, leq = 0;
                                for (uint32_t q = 0; q < cb; ++q) {
                                    const float u = cand[q];
                                    less += u < v ? 1u : 0u;
                                    leq += u <= v ? 1u : 0u;
                                }
                                if (less <= rr && rr < leq) red[5] = __float_as_uint(v);
                            }
                            __syncthreads();
                            med = __uint_as_float(red[5]);
                            done = true;
                        }
                        // a bin of more than 64 (heavy ties): the radix selection below
                    }
                }
                if (!done) {
                    // radix selection (digits of 11, 11 and 10 bits) over every
                    // workgroup's share of the distances, one barrier per digit
                    uint32_t prefix = 0, pmask = 0, rk = rank;
                    for (int pass = 0; pass < 3; ++pass) {
                        const int shift = pass == 0 ? 21 : pass == 1 ? 10 : 0;
                        const uint32_t dmask = pass == 2 ? 0x3ffu : 0x7ffu;
                        for (int q = tid; q < kBins; q += nt) hist[q] = 0;
                        __syncthreads();
                        auto count = [&](const f32x4 &Dv, bool diag) {
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const uint32_t key = __float_as_uint(fmax_(Dv[r], 0.f));
                                const bool valid = !diag || ((diag_lanes(r) >> lane) & 1ull);
                                if (valid && (key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & dmask], 1u);
                            }
                        };
                        TileWalker<K4, true> rw;
                        rw.start(X8, npad, g, col, gi * nwaves + wave, G * nwaves);
                        while (!rw.done()) {
                            f32x4 D0, D1;
                            rw.issue(X8, g, col, D0, D1);
                            count(D0, false);
                            if (rw.second()) count(D1, false);
                            rw.advance(X8, g, col);
                        }
                        rw.diagonals(X8, g, col, count);
                        __syncthreads();
                        uint32_t *rh = crhist + (long)(pass & 1) * G * kBins;
                        for (int q = tid; q < kBins; q += nt) rh[(long)gi * kBins + q] = hist[q];
                        coop_barrier(cctr, ++epoch * (uint32_t)G, a.status);
                        for (int q = tid; q < kBins; q += nt) {
                            uint32_t c = 0;
                            for (int gg = 0; gg < G; ++gg) c += rh[(long)gg * kBins + q];
                            hist[q] = c;
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
                            if (rk >= excl && rk < incl) {
                                uint32_t r2 = rk - excl;
                                for (int q = 0; q < per; ++q) {
                                    const uint32_t hq = hist[lane * per + q];
                                    if (r2 < hq) { red[0] = (uint32_t)(lane * per + q); red[1] = r2; break; }
                                    r2 -= hq;
                                }
                            }
                        }
                        __syncthreads();
                        prefix |= red[0] << shift;
                        rk = red[1];
                        pmask |= dmask << shift;
                        __syncthreads();
                    }
                    med = __uint_as_float(prefix);
                }
                med = uniform(med);
                tracker.med2 = tracker.med1;
                tracker.med1 = med;
                tracker.have = tracker.have < 2 ? tracker.have + 1 : 2;
                tracker.active = false;
                h = uniform(bandwidth_from_median(med, n, a.bw_scale));
            }
        } else if (need_median) {
            const float med = tracker.finish<K4>(X8, n, npad, WIN, hist, red);
            h = uniform(bandwidth_from_median(med, n, a.bw_scale));
        }
        if (a.h_out && tid == 0 && gi == 0) a.h_out[(long)b * a.h_stride + it] = h;
        const float beta = uniform((float)kLog2e / h);

        // (3) Stein direction
        //   phi_i = (sum_k kappa_ki v_k + c2 x_i sum_k kappa_ki) / n,
        //   v_k = s_k - c2 x_k, c2 = 2 / h
        // (the kernel-gradient term of the update folded into the score
        // rows, so one contraction of kappa with [v, 1] gives both sums).
        // The score rows become v in place; column kOne holds the 1.
        const float twob = 2.f * beta;
        const float c2 = 2.f / h;
        constexpr int NG = D <= 3 ? 1 : 2;       // row groups of four in the sums
        constexpr int kOne = NG == 1 ? 3 : 7;    // row that sums kappa
        for (int k = tid; k < npad; k += nt) {
            if (split && !COOP) {
                // the score row of particle k from the splits' partial sums
                // (rebased to their largest reference, summed in split order)
                float srow[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) srow[c] = 0.f;
                srow[7] = 1.f;
                if (k < n) {
                    float xt[D], xa[D], gr[D];
#pragma unroll
                    for (int c = 0; c < D; ++c) {
                        xt[c] = X8[(long)k * 8 + c];
                        xa[c] = xt[c] + ref[c];
                    }
                    F::grad(m, sz, mk, xa, gr);
                    if (a.trans_mode == 0) {
                        float mx = -inf;
                        for (int sp = 0; sp < L.ns_sc; ++sp)
                            mx = fmax_(mx, PART[((long)sp * ntasks * 64 + k) * kPartStride + 8]);
                        float os[8];
#pragma unroll
                        for (int c = 0; c < 8; ++c) os[c] = 0.f;
                        for (int sp = 0; sp < L.ns_sc; ++sp) {
                            const float *pp = PART + ((long)sp * ntasks * 64 + k) * kPartStride;
                            const float w = R::exp2_(pp[8] - mx);
#pragma unroll
                            for (int c = 0; c < 8; ++c) os[c] += pp[c] * w;
                        }
                        const float inv_sum = 1.f / os[7];
#pragma unroll
                        for (int c = 0; c < D; ++c) {
                            const float mb = os[c] * inv_sum * 0.5f / rs[c];
                            srow[c] = gr[c] - (xt[c] - mb) * m.inv_q[c];
                        }
                    } else {
#pragma unroll
                        for (int c = 0; c < D; ++c) srow[c] = gr[c] - (xt[c] - mbar_all[c]) * m.inv_q[c];
                    }
                }
#pragma unroll
                for (int c = 0; c < 8; ++c) S8[(long)k * 8 + c] = srow[c];
            }
#pragma unroll
            for (int c = 0; c < D; ++c) S8[(long)k * 8 + c] -= c2 * X8[(long)k * 8 + c];
            if (kOne != 7) S8[(long)k * 8 + kOne] = 1.f;
        }
        __syncthreads();
        float phi[TS][kTilesPerWave][2];  // kept in registers until every wave is done
        // source tiles [k0, k1) of this wave (split: its share of its task's)
        const int sp_st = split ? wave / ntasks : 0;
        const int k0 = split ? sp_st * nkt / L.ns_st : 0;
        const int k1 = split ? (sp_st + 1) * nkt / L.ns_st : nkt;
#pragma unroll
        for (int ts = 0; ts < TS; ++ts) {
            const int task = split ? (ts == 0 && sp_st < L.ns_st ? wave % ntasks : ntasks) : wave + ts * nwaves;
            if (task >= ntasks) break;
            const int ibase = tbase + task * 64;
            // B columns (2 beta x_i, -beta in K-row 7); the accumulator starts
            // at -beta n_i, so a Gram tile holds the exponent
            // -beta |x_k - x_i|^2 of kappa directly
            float bi0[kTilesPerWave], bi1[kTilesPerWave];
            f32x4 cb[kTilesPerWave];
            // Sums on the 4x4x1 (16-block) MFMA straight from the Gram tile
            // layout: register r of lane l holds kappa of source
            // 16 kt + 4 (l / 16) + r and target 16 q + l % 16, so block
            // b = l / 4 takes B = that register and A = rows 4 gg + l % 4 of
            // v for its source; lane l of O4[gg][q] accumulates rows
            // 4 gg + i (register i) of target 16 q + l % 16 over the source
            // quarter l / 16, summed across quarters after the pass
            f32x4 O4[NG][kTilesPerWave];
#pragma unroll
            for (int q = 0; q < kTilesPerWave; ++q) {
                const int ii = ibase + 16 * q + col;
                bi0[q] = K4 && g == 3 ? -beta : twob * X8[(long)ii * 8 + g];
                bi1[q] = g == 3 ? -beta : twob * X8[(long)ii * 8 + 4 + g];
                const float nb = -beta * X8[(long)ii * 8 + 7];
                cb[q] = f32x4{nb, nb, nb, nb};
#pragma unroll
                for (int gg = 0; gg < NG; ++gg) O4[gg][q] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
            const float *vbase = S8 + (long)(4 * g) * 8 + (lane & 3);
            // Gram tiles: A rows (x_k, n_k in the last K-row)
            const int ka = gram_col<K4>(g);
            auto gram = [&](int kt, f32x4 (&Go)[kTilesPerWave]) {
                const float *xr = X8 + (long)(kt * 16 + col) * 8;
                const float ak0 = xr[ka];
#pragma unroll
                for (int q = 0; q < kTilesPerWave; ++q) Go[q] = mfma16(ak0, bi0[q], cb[q]);
                if (!K4) {
                    const float ak1 = xr[4 + g];
#pragma unroll
                    for (int q = 0; q < kTilesPerWave; ++q) Go[q] = mfma16(ak1, bi1[q], Go[q]);
                }
            };
            // one source tile: the Gram tiles of kt + 1 are issued before the
            // exponentials of tile kt (the last tile repeats, unused); the two
            // buffers alternate
            auto tile = [&](int kt, f32x4 (&G)[kTilesPerWave], f32x4 (&Gn)[kTilesPerWave]) {
                const float *vb = vbase + (long)(kt * 16) * 8;
                float av[4][NG];
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int gg = 0; gg < NG; ++gg) av[r][gg] = vb[r * 8 + 4 * gg];
                gram(min(kt + 1, k1 - 1), Gn);
#pragma unroll
                for (int q = 0; q < kTilesPerWave; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) G[q][r] = R::exp2_(G[q][r]);
                // independent accumulators back to back
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int q = 0; q < kTilesPerWave; ++q)
#pragma unroll
                        for (int gg = 0; gg < NG; ++gg)
                            O4[gg][q] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[r][gg], G[q][r], O4[gg][q], 0, 0, 0);
            };
            f32x4 GA[kTilesPerWave], GB[kTilesPerWave];
            gram(k0, GA);
            for (int kt = k0; kt < k1; kt += 2) {
                if (kBalance) bal.step();
                tile(kt, GA, GB);
                if (kt + 1 < k1) tile(kt + 1, GB, GA);
            }
            // lane (col, g): target ibase + 16 q + col, coordinates g, 4 + g
#pragma unroll
            for (int q = 0; q < kTilesPerWave; ++q) {
                const int ii = ibase + 16 * q + col;
                const float ksum = sum_row_quarters(O4[NG - 1][q][kOne - 4 * (NG - 1)]);
                float *pp = PART + ((long)sp_st * ntasks * 64 + (ii - tbase)) * kPartStride;
                if (split && g == 0) pp[8] = ksum;
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2) {
                    const int c = g + 4 * h2;
                    float v = 0.f;
                    if (h2 < NG) {
                        // row c = 4 h2 + g: register g of the lane's row
                        const f32x4 &o = O4[h2 < NG ? h2 : 0][q];
                        const float sv = sum_quarters_scatter(o[0], o[1], o[2], o[3]);
                        if (split) {
                            if (c < D) pp[c] = sv;
                        } else if (c < D) {
                            v = (sv + c2 * X8[(long)ii * 8 + c] * ksum) * inv_n;
                        }
                    }
                    phi[ts][q][h2] = v;
                }
            }
        }
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        // the window histogram starts the next walk at zero (the barrier at
        // the end of the iteration orders this before it)
        for (int q = tid; q < 256; q += nt) whist[q] = 0;
        if (split) {
            // synchronous update from the splits' partial sums (split order):
            // the sums per (target, row) into S8 (dead after the Stein pass),
            // then per target the update and the squared norm of the moved
            // particle (the workgroup's targets; in COOP also to the exchange
            // area)
            const int ntl = ntasks * 64;
            for (int e = tid; e < ntl * 8; e += nt) {
                const int il = e >> 3, c = e & 7;
                const int cc = c < D ? c : 8;  // row 7 (or the first unused one) carries the kernel sum
                if (c < D || c == 7) {
                    float acc = 0.f;
                    for (int sp = 0; sp < L.ns_st; ++sp) acc += PART[((long)sp * ntl + il) * kPartStride + cc];
                    S8[(long)(tbase + il) * 8 + c] = acc;
                }
            }
            __syncthreads();
            for (int il = tid; il < ntl; il += nt) {
                const int i = tbase + il;
                if (i >= n) continue;
                const float ks = S8[(long)i * 8 + 7];
                float nrm = 0.f;
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    const float xc = X8[(long)i * 8 + c];
                    const float v = xc + a.step * ((S8[(long)i * 8 + c] + c2 * xc * ks) * inv_n);
                    X8[(long)i * 8 + c] = v;
                    nrm += v * v;
                }
                X8[(long)i * 8 + 7] = nrm;
                if (COOP)
#pragma unroll
                    for (int c = 0; c < 8; ++c) cX[(long)i * 8 + c] = X8[(long)i * 8 + c];
            }
        }
        // synchronous update, then unscaled squared norms for the next median
#pragma unroll
        for (int ts = 0; ts < TS; ++ts) {
            const int task = wave + ts * nwaves;
            if (split || task >= ntasks) break;
#pragma unroll
            for (int q = 0; q < kTilesPerWave; ++q) {
                const int ii = task * 64 + 16 * q + col;
                if (ii < n) {
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2) {
                        const int c = g + 4 * h2;
                        if (c < D) X8[(long)ii * 8 + c] += a.step * phi[ts][q][h2];
                    }
                }
            }
        }
        // a wave's particles were written by its own lanes only
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int ts = 0; ts < TS; ++ts) {
            const int task = wave + ts * nwaves;
            if (split || task >= ntasks) break;
            const int i = task * 64 + lane;
            if (i < n) {
                float nrm = 0.f;
#pragma unroll
                for (int c = 0; c < D; ++c) { const float v = X8[(long)i * 8 + c]; nrm += v * v; }
                X8[(long)i * 8 + 7] = nrm;
            }
        }
        __syncthreads();
        if constexpr (COOP) {
            // every workgroup's moved particles
            coop_barrier(cctr, ++epoch * (uint32_t)G, a.status);
            for (int i = tid; i < n; i += nt)
#pragma unroll
                for (int c = 0; c < 8; ++c) X8[(long)i * 8 + c] = cX[(long)i * 8 + c];
            __syncthreads();
        }
    }

    bool bad = false;
    const int i_lo = COOP ? tbase : 0, i_hi = COOP ? min(n, tbase + ntasks * 64) : n;
    for (int i = i_lo + tid; a.do_svgd && i < i_hi; i += nt) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const float v = X8[(long)i * 8 + c] + ref[c];
            bad |= !R::finite(v);
            xg[(long)i * D + c] = v;
        }
    }

    if (a.do_viterbi) {
        for (int j = tid; j < np; j += nt) PHP[j] = a.phi_prev ? a.phi_prev[(long)b * a.phi_prev_stride + j] : 0.f;
        __syncthreads();
        for (int i = i_lo + tid; i < i_hi; i += nt) {
            float xs[D], xa[D];
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const float xt = X8[(long)i * 8 + c];
                xs[c] = xt * rs[c];
                xa[c] = xt + ref[c];
            }
            ArgBest<float> ab{-inf, -inf, 0};
            bool nan_seen = false;
            for (int j = 0; j < np; ++j) {
                float q2 = 0.f;
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    const float r = xs[c] - 0.5f * VT[(long)c * nppad + j];
                    q2 += r * r;
                }
                const float A = m.log_z - (float)kLn2 * q2;
                const float cij = A + PHP[j];
                nan_seen |= (cij != cij);
                if (j == 0) { ab.best = cij; ab.arg = 0; }
                else argbest_push(ab, cij, j);
            }
            const float ell = F::loglik(m, sz, mk, xa);
            const float ph = ab.best + ell;
            nan_seen |= (ph != ph);
            bad |= nan_seen;
            a.phi[(long)b * a.phi_stride + i] = ph;
            a.psi[(long)b * a.psi_stride + i] = ab.arg;
            if (a.flags) {
                const float mag = ab.best < 0 ? -ab.best : ab.best;
                const float sc_ = mag > 1.f ? mag : 1.f;
                a.flags[(long)b * a.flags_stride + i] = (np > 1 && ab.second >= ab.best - a.tie_tol * sc_) ? 1 : 0;
            }
        }
    }
    if (bad) atomicOr(a.status, STATUS_NONFINITE);
}

template <int KIND, int D, bool SPLIT>
__global__ __launch_bounds__(kMaxWaves * 64) void k_step_mfma(StepArgs<float> a)
{
    step_mfma_body<KIND, D, kMaxParticles / 64 / kMaxWaves, SPLIT>(a, blockIdx.x);
}

// Multi-workgroup step: workgroup blockIdx.x is group blockIdx.x % G of
// sequence blockIdx.x / G (a cooperative launch: all resident at once).
template <int KIND, int D>
__global__ __launch_bounds__(kMaxWaves * 64) void k_step_mfma_coop(StepArgs<float> a, CoopArgs c)
{
    c.gi = (int)(blockIdx.x % (unsigned)c.G);
    step_mfma_body<KIND, D, 1, true, true>(a, (int)(blockIdx.x / (unsigned)c.G), c);
}

} // namespace smsq
