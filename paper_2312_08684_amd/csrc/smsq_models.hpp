// Model families as device functions: transition mean f_t, observation
// log-likelihood log p(z | x) and its analytic gradient in x (paper Sec. II,
// eq. SSM; scenario shapes of Sec. V).  The transition density of every family
// is Gaussian, N(f_t(x_{t-1}), diag(q)); the kernels evaluate it themselves.
#pragma once

#include "smsq_common.hpp"

namespace smsq {

enum Kind { GROWTH1D = 0, RANGE2D = 1, CV4D = 2, ARM7 = 3, LINGAUSS = 4, SE2 = 5, ARM14 = 6 };

// Per-launch model constants, precomputed on the host in the kernel's type.
template <typename T> struct DevModel {
    int kind, d, obs_dim, n_obs;
    T q[16];       // transition variances
    T inv_q[16];   // 1 / q
    T sqrt_q[16];  // sqrt(q)
    T rs[16];      // sqrt(log2(e) / (2 q)): x * rs puts -(x-m)^2/(2q) in log2 units
    T log_z;       // -1/2 sum_d log(2 pi q_d)
    T p[64];       // family parameters
    T aux[16];     // family constants (RANGE2D: 1/r_var; ARM7: cos alpha_i, sin alpha_i;
                   // SE2: 1/r_var, 1/b_var, log-density constant of one landmark)
    double grow[3]; // GROWTH1D cosine term c, omega, phase; ARM14 input amplitude,
                    // frequency, phase step (kept in double)
};

template <typename T, int KIND, int D> struct Family;

// ---------------------------------------------------------------------------
template <typename T> struct Family<T, GROWTH1D, 1> {
    static __device__ void mean(const DevModel<T> &m, int t, const T *x, T *out)
    {
        const T v = x[0];
        const T c = (T)(m.grow[0] * cos(m.grow[1] * (double)t + m.grow[2]));
        out[0] = m.p[0] * v + m.p[1] * v / ((T)1 + v * v) + c;
    }
    static __device__ T loglik(const DevModel<T> &m, const T *z, const uint8_t *mask, const T *x)
    {
        if (mask && !mask[0]) return (T)0;
        const T r = z[0] - m.p[5] * x[0] * x[0];
        return (T)-0.5 * r * r / m.p[6] - (T)0.5 * RealOps<T>::log_((T)(2.0 * kPi) * m.p[6]);
    }
    static __device__ void grad(const DevModel<T> &m, const T *z, const uint8_t *mask, const T *x, T *g)
    {
        g[0] = (T)0;
        if (mask && !mask[0]) return;
        const T r = z[0] - m.p[5] * x[0] * x[0];
        g[0] = r / m.p[6] * ((T)2 * m.p[5] * x[0]);
    }
};

// ---------------------------------------------------------------------------
template <typename T> struct Family<T, RANGE2D, 2> {
    static __device__ void mean(const DevModel<T> &, int, const T *x, T *out)
    {
        out[0] = x[0];
        out[1] = x[1];
    }
    static __device__ T loglik(const DevModel<T> &m, const T *z, const uint8_t *mask, const T *x)
    {
        const int nb = m.n_obs;
        const T lc = (T)0.5 * RealOps<T>::log_((T)(2.0 * kPi) * m.p[0]);
        T s = 0;
        for (int b = 0; b < nb; ++b) {
            if (mask && !mask[b]) continue;
            const T dx = x[0] - m.p[2 + 2 * b], dy = x[1] - m.p[3 + 2 * b];
            const T e = z[b] - RealOps<T>::sqrt_(dx * dx + dy * dy);
            s += (T)-0.5 * e * e / m.p[0] - lc;
        }
        return s;
    }
    static __device__ void grad(const DevModel<T> &m, const T *z, const uint8_t *mask, const T *x, T *g)
    {
        g[0] = g[1] = (T)0;
        for (int b = 0; b < m.n_obs; ++b) {
            if (mask && !mask[b]) continue;
            const T dx = x[0] - m.p[2 + 2 * b], dy = x[1] - m.p[3 + 2 * b];
            const T r = RealOps<T>::sqrt_(dx * dx + dy * dy);
            if (r < (T)1e-12) continue;
            const T w = (z[b] - r) * m.aux[0] / r;  // aux[0] = 1 / r_var
            g[0] += w * dx;
            g[1] += w * dy;
        }
    }
};

// ---------------------------------------------------------------------------
// Detection / clutter mixture: p(Z|x) = V^-(M-1) [(1-P_D)/V + (P_D/M) sum_m
// N(z_m; (px,py), r I)].  Evaluated as a running-max log-sum-exp over the
// clutter term and the M detection terms.
template <typename T> struct Family<T, CV4D, 4> {
    static __device__ void mean(const DevModel<T> &m, int, const T *x, T *out)
    {
        out[0] = x[0] + m.p[0] * x[2];
        out[1] = x[1] + m.p[0] * x[3];
        out[2] = x[2];
        out[3] = x[3];
    }
    static __device__ int count(const DevModel<T> &m, const uint8_t *mask)
    {
        int M = 0;
        for (int k = 0; k < m.n_obs; ++k) M += (mask == nullptr || mask[k]) ? 1 : 0;
        return M;
    }
    // Running log-sum-exp: returns (mx, s) with log sum = mx + log s, and the
    // responsibility-weighted residual sums gx, gy (scaled like s).
    static __device__ void accumulate(const DevModel<T> &m, const T *z, const uint8_t *mask, const T *x,
                                      int M, T &mx, T &s, T &gx, T &gy)
    {
        const T rv = m.p[1], pd = m.p[2], V = m.p[3];
        mx = RealOps<T>::log_(((T)1 - pd) / V);
        s = (T)1;
        gx = gy = (T)0;
        const T ldet = RealOps<T>::log_(pd / (T)M) - RealOps<T>::log_((T)(2.0 * kPi) * rv);
        for (int k = 0; k < m.n_obs; ++k) {
            if (mask && !mask[k]) continue;
            const T ex = z[2 * k] - x[0], ey = z[2 * k + 1] - x[1];
            const T v = ldet - (T)0.5 * (ex * ex + ey * ey) / rv;
            if (v > mx) {
                const T sf = RealOps<T>::exp_(mx - v);
                s = s * sf + (T)1;
                gx = gx * sf + ex;
                gy = gy * sf + ey;
                mx = v;
            } else {
                const T e = RealOps<T>::exp_(v - mx);
                s += e;
                gx += e * ex;
                gy += e * ey;
            }
        }
    }
    static __device__ T loglik(const DevModel<T> &m, const T *z, const uint8_t *mask, const T *x)
    {
        const int M = count(m, mask);
        if (M == 0) return RealOps<T>::log_((T)1 - m.p[2]);
        T mx, s, gx, gy;
        accumulate(m, z, mask, x, M, mx, s, gx, gy);
        return -(T)(M - 1) * RealOps<T>::log_(m.p[3]) + mx + RealOps<T>::log_(s);
    }
    static __device__ void grad(const DevModel<T> &m, const T *z, const uint8_t *mask, const T *x, T *g)
    {
        g[0] = g[1] = g[2] = g[3] = (T)0;
        const int M = count(m, mask);
        if (M == 0) return;
        T mx, s, gx, gy;
        accumulate(m, z, mask, x, M, mx, s, gx, gy);
        const T sc = (T)1 / (s * m.p[1]);
        g[0] = gx * sc;
        g[1] = gy * sc;
    }
};

// ---------------------------------------------------------------------------
// Standard-DH 7-joint chain; the gradient is J^T (z - p) / r with the
// geometric Jacobian column z_{i-1} x (p - o_{i-1}) of each revolute joint.
// Two forward sweeps: the first finds the end-effector position p, the
// second rebuilds each frame (from the cached sines / cosines) and
// accumulates the Jacobian-transpose product, so no frame is stored.
template <typename T> struct Family<T, ARM7, 7> {
    static __device__ void mean(const DevModel<T> &, int, const T *x, T *out)
    {
#pragma unroll
        for (int a = 0; a < 7; ++a) out[a] = x[a];
    }
    struct Frame {
        T R00, R01, R02, R10, R11, R12, R20, R21, R22, o0, o1, o2;
        __device__ void reset()
        {
            R00 = 1; R01 = 0; R02 = 0; R10 = 0; R11 = 1; R12 = 0; R20 = 0; R21 = 0; R22 = 1;
            o0 = o1 = o2 = 0;
        }
        // frame <- frame * A_i with A_i = Rz(q) Tz(dd) Tx(a) Rx(alpha)
        __device__ void advance(T ct, T st, T ca, T sa, T a, T dd)
        {
            const T A00 = ct, A01 = -st * ca, A02 = st * sa;
            const T A10 = st, A11 = ct * ca, A12 = -ct * sa;
            const T A21 = sa, A22 = ca;
            const T t0 = a * ct, t1 = a * st, t2 = dd;
            o0 += R00 * t0 + R01 * t1 + R02 * t2;
            o1 += R10 * t0 + R11 * t1 + R12 * t2;
            o2 += R20 * t0 + R21 * t1 + R22 * t2;
            const T n00 = R00 * A00 + R01 * A10, n01 = R00 * A01 + R01 * A11 + R02 * A21,
                    n02 = R00 * A02 + R01 * A12 + R02 * A22;
            const T n10 = R10 * A00 + R11 * A10, n11 = R10 * A01 + R11 * A11 + R12 * A21,
                    n12 = R10 * A02 + R11 * A12 + R12 * A22;
            const T n20 = R20 * A00 + R21 * A10, n21 = R20 * A01 + R21 * A11 + R22 * A21,
                    n22 = R20 * A02 + R21 * A12 + R22 * A22;
            R00 = n00; R01 = n01; R02 = n02;
            R10 = n10; R11 = n11; R12 = n12;
            R20 = n20; R21 = n21; R22 = n22;
        }
    };
    static __device__ void end_effector(const DevModel<T> &m, const T *q, T *st, T *ct, T *p)
    {
        Frame f;
        f.reset();
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            RealOps<T>::sincos_(q[i], &st[i], &ct[i]);
            f.advance(ct[i], st[i], m.aux[i], m.aux[7 + i], m.p[1 + i], m.p[15 + i]);
        }
        p[0] = f.o0; p[1] = f.o1; p[2] = f.o2;
    }
    static __device__ T loglik(const DevModel<T> &m, const T *z, const uint8_t *mask, const T *x)
    {
        if (mask && !mask[0]) return (T)0;
        T st[7], ct[7], p[3];
        end_effector(m, x, st, ct, p);
        const T e0 = z[0] - p[0], e1 = z[1] - p[1], e2 = z[2] - p[2];
        return (T)-0.5 * (e0 * e0 + e1 * e1 + e2 * e2) / m.p[0]
               - (T)1.5 * RealOps<T>::log_((T)(2.0 * kPi) * m.p[0]);
    }
    static __device__ void grad(const DevModel<T> &m, const T *z, const uint8_t *mask, const T *x, T *g)
    {
#pragma unroll
        for (int a = 0; a < 7; ++a) g[a] = (T)0;
        if (mask && !mask[0]) return;
        T st[7], ct[7], p[3];
        end_effector(m, x, st, ct, p);
        const T ir = (T)1 / m.p[0];
        const T e0 = (z[0] - p[0]) * ir, e1 = (z[1] - p[1]) * ir, e2 = (z[2] - p[2]) * ir;
        Frame f;
        f.reset();
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            // joint i+1 turns about the z axis of frame i through its origin
            const T v0 = p[0] - f.o0, v1 = p[1] - f.o1, v2 = p[2] - f.o2;
            const T z0 = f.R02, z1 = f.R12, z2 = f.R22;
            const T c0 = z1 * v2 - z2 * v1;
            const T c1 = z2 * v0 - z0 * v2;
            const T c2 = z0 * v1 - z1 * v0;
            g[i] = c0 * e0 + c1 * e1 + c2 * e2;
            f.advance(ct[i], st[i], m.aux[i], m.aux[7 + i], m.p[1 + i], m.p[15 + i]);
        }
    }
};

// ---------------------------------------------------------------------------
// 14-D manipulator of Sec. V-D, x = [q; qdot]: q_t = q + qdot dt and
// qdot_t = qdot + u_{t-1} dt with u_{t-1,i} = amp sin(freq (t - 1) + phase_step i).
// The observation is the end effector of the same DH chain as ARM7, whose
// constants sit at the same parameter slots: the likelihood and its
// joint-angle gradient are ARM7's, the velocity gradient is zero.
template <typename T> struct Family<T, ARM14, 14> {
    using Arm = Family<T, ARM7, 7>;
    static __device__ void mean(const DevModel<T> &m, int t, const T *x, T *out)
    {
        const T dt = m.p[22];
#pragma unroll
        for (int a = 0; a < 7; ++a) {
            const T u = (T)(m.grow[0] * sin(m.grow[1] * (double)(t - 1) + m.grow[2] * (double)a));
            out[a] = x[a] + x[7 + a] * dt;
            out[7 + a] = x[7 + a] + u * dt;
        }
    }
    static __device__ T loglik(const DevModel<T> &m, const T *z, const uint8_t *mask, const T *x)
    {
        return Arm::loglik(m, z, mask, x);
    }
    static __device__ void grad(const DevModel<T> &m, const T *z, const uint8_t *mask, const T *x, T *g)
    {
        Arm::grad(m, z, mask, x, g);
#pragma unroll
        for (int a = 7; a < 14; ++a) g[a] = (T)0;
    }
};

// ---------------------------------------------------------------------------
// SE(2) pose (px, py, heading) of Sec. V-B: the heading turns by omega dt and
// the position moves v dt along the new heading.  One range-bearing
// measurement per step from one of n_l landmarks whose identity is unknown:
// the likelihood is the equal-weight mixture over the landmarks, evaluated as
// a running-max log-sum-exp in one pass (the gradient is the
// responsibility-weighted sum of the per-landmark gradients, accumulated in
// the same pass).  The bearing residual is mapped into [-pi, pi).
template <typename T> struct Family<T, SE2, 3> {
    static __device__ void mean(const DevModel<T> &m, int, const T *x, T *out)
    {
        const T th = x[2] + m.p[2] * m.p[0];
        T s, c;
        RealOps<T>::sincos_(th, &s, &c);
        const T vdt = m.p[1] * m.p[0];
        out[0] = x[0] + vdt * c;
        out[1] = x[1] + vdt * s;
        out[2] = th;
    }
    static __device__ T wrap(T a)
    {
        const T tau = (T)(2.0 * kPi);
        return a - tau * RealOps<T>::floor_((a + (T)kPi) / tau);
    }
    // log-mixture and, with g != nullptr, its gradient in (px, py)
    static __device__ T mixture(const DevModel<T> &m, const T *z, const T *x, T *g)
    {
        const int nl = (int)m.p[5];
        T mx = -RealOps<T>::inf(), s = 0, g0 = 0, g1 = 0;
        for (int l = 0; l < nl; ++l) {
            const T dx = x[0] - m.p[6 + 2 * l], dy = x[1] - m.p[7 + 2 * l];
            const T r2 = dx * dx + dy * dy;
            const T rho = RealOps<T>::sqrt_(r2);
            const T er = z[0] - rho;
            const T eb = wrap(z[1] - RealOps<T>::atan2_(dy, dx));
            const T tl = (T)-0.5 * (er * er * m.aux[0] + eb * eb * m.aux[1]);
            T l0 = 0, l1 = 0;
            if (g && rho >= (T)1e-12) {
                const T gr = er * m.aux[0] / rho, gb = eb * m.aux[1] / r2;
                l0 = gr * dx - gb * dy;
                l1 = gr * dy + gb * dx;
            }
            if (tl > mx) {
                const T sc = RealOps<T>::exp_(mx - tl);
                s = s * sc + (T)1;
                g0 = g0 * sc + l0;
                g1 = g1 * sc + l1;
                mx = tl;
            } else {
                const T w = RealOps<T>::exp_(tl - mx);
                s += w;
                g0 += w * l0;
                g1 += w * l1;
            }
        }
        if (g) {
            g[0] = g0 / s;
            g[1] = g1 / s;
        }
        return mx + RealOps<T>::log_(s) + m.aux[2];
    }
    static __device__ T loglik(const DevModel<T> &m, const T *z, const uint8_t *mask, const T *x)
    {
        if (mask && !mask[0]) return (T)0;
        return mixture(m, z, x, nullptr);
    }
    static __device__ void grad(const DevModel<T> &m, const T *z, const uint8_t *mask, const T *x, T *g)
    {
        g[0] = g[1] = g[2] = (T)0;
        if (mask && !mask[0]) return;
        mixture(m, z, x, g);
    }
};

// ---------------------------------------------------------------------------
template <typename T, int D> struct Family<T, LINGAUSS, D> {
    static __device__ void mean(const DevModel<T> &m, int, const T *x, T *out)
    {
#pragma unroll
        for (int a = 0; a < D; ++a) {
            T s = 0;
#pragma unroll
            for (int b = 0; b < D; ++b) s += m.p[a * D + b] * x[b];
            out[a] = s;
        }
    }
    static __device__ T loglik(const DevModel<T> &m, const T *z, const uint8_t *mask, const T *x)
    {
        if (mask && !mask[0]) return (T)0;
        T s = 0;
        for (int r = 0; r < m.obs_dim; ++r) {
            T hx = 0;
#pragma unroll
            for (int c = 0; c < D; ++c) hx += m.p[16 + r * D + c] * x[c];
            const T e = z[r] - hx;
            s += (T)-0.5 * e * e / m.p[32 + r] - (T)0.5 * RealOps<T>::log_((T)(2.0 * kPi) * m.p[32 + r]);
        }
        return s;
    }
    static __device__ void grad(const DevModel<T> &m, const T *z, const uint8_t *mask, const T *x, T *g)
    {
#pragma unroll
        for (int c = 0; c < D; ++c) g[c] = (T)0;
        if (mask && !mask[0]) return;
        for (int r = 0; r < m.obs_dim; ++r) {
            T hx = 0;
#pragma unroll
            for (int c = 0; c < D; ++c) hx += m.p[16 + r * D + c] * x[c];
            const T w = (z[r] - hx) / m.p[32 + r];
#pragma unroll
            for (int c = 0; c < D; ++c) g[c] += m.p[16 + r * D + c] * w;
        }
    }
};

} // namespace smsq
