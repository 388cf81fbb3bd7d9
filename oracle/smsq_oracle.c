/*
 * Stein-MAP-Seq CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, scalar FP64 implementation of what the MI355X hot path
 * computes, written from the paper (Seo & Kia, "A Computationally Efficient
 * Maximum A Posteriori Sequence Estimation via Stein Variational Inference",
 * arXiv 2312.08684).  Only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product path never does.  It shares no
 * source with the HIP library: its model log-densities, random-number
 * generator, median, score, Stein update, forward recursion and backtracking
 * are all written out here on their own.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -fopenmp (no fast-math), so
 * that every floating-point operation is a single IEEE double operation in
 * source order.  OpenMP splits only the loops over particles (each particle's
 * sums keep their order) and the sort of the median (a sorted array is the
 * same however it is sorted), so any thread count gives bit-identical
 * results; or_set_threads picks the count.
 *
 * Section / equation map (paper numbering):
 *   models           Sec. II, eq. (SSM); scenario models of Sec. V (the
 *                    SE(2) pose with unknown landmark identity is Sec. V-B,
 *                    the 14-D second-order manipulator Sec. V-D)
 *   or_philox*       counter-based RNG (Salmon et al., SC'11), used only for
 *                    the predictive initial particles
 *   or_bandwidth     RBF kernel with the median-heuristic bandwidth (Sec. V
 *                    set-up; the formula h = med / ln N follows SVGD's
 *                    original heuristic, Liu & Wang 2016, cited by the paper)
 *   or_scores        score of the per-step target p(z_t, x_t | x_{t-1}) under
 *                    the particle mixture of the previous step (Lemma IV.3,
 *                    eq. SVGD_newupdate; trans_mode 0 takes the gradient of
 *                    log sum_j w_j p(x | x_{t-1}^j), trans_mode 1 the paper's
 *                    literal average of the per-j gradients)
 *   or_stein_phi     Stein direction of eq. SVGD_newupdate / svgd_iterate, with
 *                    the RBF kernel or the IMQ and Matern kernels of the
 *                    kernel ablation (Sec. V-E, Table VIII)
 *   or_svgd_step     Algorithm 2 steps 1) and 2): x <- x + eps * phi, L times
 *   or_viterbi_*     forward recursion, eq. forward_recursion
 *   or_backtrack     backtracking of Sec. IV-B / Algorithm 2 step 4)
 *   or_path_score    trajectory score J(s) of Theorem IV.1
 *   or_run_sequence  Algorithm 2 end to end (weights 1: the previous step's
 *                    forward-recursion scores as the mixture log-weights,
 *                    w_j proportional to exp(phi_{t-1}(j)))
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXD 16

enum { OR_GROWTH1D = 0, OR_RANGE2D = 1, OR_CV4D = 2, OR_ARM7 = 3, OR_LINGAUSS = 4, OR_SE2 = 5, OR_ARM14 = 6 };
enum { OR_OK = 0, OR_INVALID = 1, OR_NONFINITE = 4 };

typedef struct {
    int kind, d, obs_dim, n_obs;
    double q_var[16];
    double params[64];
} or_model;

static const double OR_PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): 10 rounds of two 32x32->64 multiplies, with the */
/* key bumped by the Weyl constants between rounds.                          */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* d (<= 16) standard normals for particle i at step t of sequence seq.
 * Counter (i, t, seq, block), key (seed low word, seed high word); block b
 * gives uniforms 4b..4b+3, each (u + 0.5) * 2^-32, and consecutive pairs go
 * through Box-Muller in FP64.  Blocks are drawn as far as the pairs need, so
 * the first eight normals are the same for every d. */
void or_normals(uint64_t seed, uint32_t seq, uint32_t t, uint32_t i, int d, double *out)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    double u[16];
    int pairs = (d + 1) / 2;
    for (int blk = 0; 4 * blk < 2 * pairs; ++blk) {
        uint32_t ctr[4] = { i, t, seq, (uint32_t)blk };
        uint32_t r[4];
        or_philox4x32_10(ctr, key, r);
        for (int q = 0; q < 4; ++q) u[4 * blk + q] = ((double)r[q] + 0.5) * (1.0 / 4294967296.0);
    }
    for (int p = 0; p < pairs; ++p) {
        double rad = sqrt(-2.0 * log(u[2 * p]));
        double ang = 2.0 * OR_PI * u[2 * p + 1];
        out[2 * p] = rad * cos(ang);
        if (2 * p + 1 < d) out[2 * p + 1] = rad * sin(ang);
    }
}

/* ------------------------------------------------------------------------ */
/* Models: transition mean f_t, Gaussian transition log-density, observation */
/* log-likelihood and its gradient in x.                                     */
/* ------------------------------------------------------------------------ */
void or_transition_mean(const or_model *m, int t, const double *x, double *out)
{
    const double *p = m->params;
    int d = m->d;
    switch (m->kind) {
    case OR_GROWTH1D: {
        double v = x[0];
        out[0] = p[0] * v + p[1] * v / (1.0 + v * v) + p[2] * cos(p[3] * (double)t + p[4]);
        break;
    }
    case OR_CV4D:
        out[0] = x[0] + p[0] * x[2];
        out[1] = x[1] + p[0] * x[3];
        out[2] = x[2];
        out[3] = x[3];
        break;
    case OR_LINGAUSS:
        for (int a = 0; a < d; ++a) {
            double s = 0.0;
            for (int b = 0; b < d; ++b) s += p[a * d + b] * x[b];
            out[a] = s;
        }
        break;
    case OR_SE2: {
        /* Sec. V-B pose model: the heading turns by omega dt, then the
         * position moves v dt along the new heading theta_t */
        double th = x[2] + p[2] * p[0];
        out[0] = x[0] + p[1] * p[0] * cos(th);
        out[1] = x[1] + p[1] * p[0] * sin(th);
        out[2] = th;
        break;
    }
    case OR_ARM14: {
        /* Sec. V-D second-order joints: q_t = q + qdot dt, qdot_t = qdot +
         * u_{t-1} dt with u_{t-1,i} = amp sin(freq (t - 1) + phase_step i) */
        double dt = p[22], amp = p[23], freq = p[24], ph = p[25];
        for (int a = 0; a < 7; ++a) {
            out[a] = x[a] + x[7 + a] * dt;
            out[7 + a] = x[7 + a] + amp * sin(freq * (double)(t - 1) + ph * (double)a) * dt;
        }
        break;
    }
    default: /* random walks: range2d, arm7 */
        for (int a = 0; a < d; ++a) out[a] = x[a];
    }
}

/* log N(x; mean, diag(q_var)), with its normalising constant. */
double or_log_transition(const or_model *m, const double *x, const double *mean)
{
    double quad = 0.0, logdet = 0.0;
    for (int a = 0; a < m->d; ++a) {
        double r = x[a] - mean[a];
        quad += r * r / m->q_var[a];
        logdet += log(2.0 * OR_PI * m->q_var[a]);
    }
    return -0.5 * quad - 0.5 * logdet;
}

/* Standard-DH forward kinematics with the frame origins and z axes that the
 * geometric Jacobian needs: frame i = A_1 ... A_i, A_i = Rz(q_i) Tz(d_i)
 * Tx(a_i) Rx(alpha_i). */
static void arm_frames(const or_model *m, const double *q, double org[8][3], double zax[8][3])
{
    const double *la = m->params + 1, *al = m->params + 8, *ld = m->params + 15;
    double R[3][3] = { {1, 0, 0}, {0, 1, 0}, {0, 0, 1} };
    double o[3] = { 0, 0, 0 };
    for (int c = 0; c < 3; ++c) { org[0][c] = 0.0; zax[0][c] = R[c][2]; }
    for (int i = 0; i < 7; ++i) {
        double ct = cos(q[i]), st = sin(q[i]), ca = cos(al[i]), sa = sin(al[i]);
        double A[3][3] = { { ct, -st * ca,  st * sa },
                           { st,  ct * ca, -ct * sa },
                           { 0.0, sa,       ca      } };
        double tr[3] = { la[i] * ct, la[i] * st, ld[i] };
        double Rn[3][3], on[3];
        for (int r = 0; r < 3; ++r) {
            on[r] = o[r];
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int k = 0; k < 3; ++k) s += R[r][k] * A[k][c];
                Rn[r][c] = s;
                on[r] += R[r][c] * tr[c];
            }
        }
        memcpy(R, Rn, sizeof R);
        memcpy(o, on, sizeof o);
        for (int c = 0; c < 3; ++c) { org[i + 1][c] = o[c]; zax[i + 1][c] = R[c][2]; }
    }
}

void or_arm_fk(const or_model *m, const double *q, double *pos)
{
    double org[8][3], zax[8][3];
    arm_frames(m, q, org, zax);
    for (int c = 0; c < 3; ++c) pos[c] = org[7][c];
}

static int obs_on(const uint8_t *mask, int o) { return mask == NULL || mask[o] != 0; }

/* Angle mapped into [-pi, pi): a - 2 pi floor((a + pi) / (2 pi)). */
double or_wrap_angle(double a) { return a - 2.0 * OR_PI * floor((a + OR_PI) / (2.0 * OR_PI)); }

/* Sec. V-B association-marginalised likelihood.  For landmark l at Gamma_l:
 * term_l = log p(l) + log N(z_r; |P - Gamma_l|, r_var)
 *        + log N(wrap(z_b - atan2(y - Gamma_l,y, x - Gamma_l,x)); 0, b_var),
 * p(l) = 1 / n_l.  Fills terms[l] and the offsets and residuals per landmark. */
static void se2_terms(const double *p, const double *z, const double *x, double *terms,
                      double *dx, double *dy, double *rho, double *er, double *eb)
{
    int nl = (int)p[5];
    for (int l = 0; l < nl; ++l) {
        dx[l] = x[0] - p[6 + 2 * l];
        dy[l] = x[1] - p[7 + 2 * l];
        rho[l] = sqrt(dx[l] * dx[l] + dy[l] * dy[l]);
        er[l] = z[0] - rho[l];
        eb[l] = or_wrap_angle(z[1] - atan2(dy[l], dx[l]));
        terms[l] = -log((double)nl) - 0.5 * er[l] * er[l] / p[3] - 0.5 * log(2.0 * OR_PI * p[3])
                   - 0.5 * eb[l] * eb[l] / p[4] - 0.5 * log(2.0 * OR_PI * p[4]);
    }
}

double or_loglik(const or_model *m, const double *z, const uint8_t *mask, const double *x)
{
    const double *p = m->params;
    switch (m->kind) {
    case OR_GROWTH1D: {
        if (!obs_on(mask, 0)) return 0.0;
        double r = z[0] - p[5] * x[0] * x[0];
        return -0.5 * r * r / p[6] - 0.5 * log(2.0 * OR_PI * p[6]);
    }
    case OR_RANGE2D: {
        int nb = (int)p[1];
        double s = 0.0;
        for (int b = 0; b < nb; ++b) {
            if (!obs_on(mask, b)) continue;
            double dx = x[0] - p[2 + 2 * b], dy = x[1] - p[3 + 2 * b];
            double r = sqrt(dx * dx + dy * dy);
            double e = z[b] - r;
            s += -0.5 * e * e / p[0] - 0.5 * log(2.0 * OR_PI * p[0]);
        }
        return s;
    }
    case OR_CV4D: {
        /* p(Z|x) = V^-(M-1) [ (1-P_D)/V + (P_D/M) sum_m N(z_m; Hx, r I) ] */
        double dt = p[0], rv = p[1], pd = p[2], V = p[3];
        (void)dt;
        int M = 0;
        for (int k = 0; k < m->n_obs; ++k) M += obs_on(mask, k);
        if (M == 0) return log(1.0 - pd);
        double terms[17];
        int nt = 0;
        terms[nt++] = log((1.0 - pd) / V);
        for (int k = 0; k < m->n_obs; ++k) {
            if (!obs_on(mask, k)) continue;
            double ex = z[2 * k] - x[0], ey = z[2 * k + 1] - x[1];
            terms[nt++] = log(pd / (double)M) - 0.5 * (ex * ex + ey * ey) / rv
                          - log(2.0 * OR_PI * rv);
        }
        double mx = terms[0];
        for (int k = 1; k < nt; ++k) if (terms[k] > mx) mx = terms[k];
        double s = 0.0;
        for (int k = 0; k < nt; ++k) s += exp(terms[k] - mx);
        return -(double)(M - 1) * log(V) + mx + log(s);
    }
    case OR_ARM7:
    case OR_ARM14: { /* the end effector depends on the joint angles x[0..7) only */
        if (!obs_on(mask, 0)) return 0.0;
        double pos[3];
        or_arm_fk(m, x, pos);
        double q = 0.0;
        for (int c = 0; c < 3; ++c) { double e = z[c] - pos[c]; q += e * e; }
        return -0.5 * q / p[0] - 1.5 * log(2.0 * OR_PI * p[0]);
    }
    case OR_SE2: {
        if (!obs_on(mask, 0)) return 0.0;
        int nl = (int)p[5];
        double terms[8], dx[8], dy[8], rho[8], er[8], eb[8];
        se2_terms(p, z, x, terms, dx, dy, rho, er, eb);
        double mx = terms[0];
        for (int l = 1; l < nl; ++l) if (terms[l] > mx) mx = terms[l];
        double s = 0.0;
        for (int l = 0; l < nl; ++l) s += exp(terms[l] - mx);
        return mx + log(s);
    }
    case OR_LINGAUSS: {
        if (!obs_on(mask, 0)) return 0.0;
        int d = m->d, o = m->obs_dim;
        double s = 0.0;
        for (int r = 0; r < o; ++r) {
            double hx = 0.0;
            for (int c = 0; c < d; ++c) hx += p[16 + r * d + c] * x[c];
            double e = z[r] - hx;
            s += -0.5 * e * e / p[32 + r] - 0.5 * log(2.0 * OR_PI * p[32 + r]);
        }
        return s;
    }
    }
    return NAN;
}

void or_grad_loglik(const or_model *m, const double *z, const uint8_t *mask, const double *x, double *g)
{
    const double *p = m->params;
    int d = m->d;
    for (int a = 0; a < d; ++a) g[a] = 0.0;
    switch (m->kind) {
    case OR_GROWTH1D:
        if (obs_on(mask, 0)) {
            double r = z[0] - p[5] * x[0] * x[0];
            g[0] = r / p[6] * (2.0 * p[5] * x[0]);
        }
        break;
    case OR_RANGE2D: {
        int nb = (int)p[1];
        for (int b = 0; b < nb; ++b) {
            if (!obs_on(mask, b)) continue;
            double dx = x[0] - p[2 + 2 * b], dy = x[1] - p[3 + 2 * b];
            double r = sqrt(dx * dx + dy * dy);
            if (r < 1e-12) continue;
            double w = (z[b] - r) / p[0] / r;
            g[0] += w * dx;
            g[1] += w * dy;
        }
        break;
    }
    case OR_CV4D: {
        double rv = p[1], pd = p[2], V = p[3];
        int M = 0;
        for (int k = 0; k < m->n_obs; ++k) M += obs_on(mask, k);
        if (M == 0) break;
        /* responsibilities of the clutter term and of each detection */
        double terms[17];
        int idx[17];
        int nt = 0;
        terms[nt] = log((1.0 - pd) / V); idx[nt++] = -1;
        for (int k = 0; k < m->n_obs; ++k) {
            if (!obs_on(mask, k)) continue;
            double ex = z[2 * k] - x[0], ey = z[2 * k + 1] - x[1];
            terms[nt] = log(pd / (double)M) - 0.5 * (ex * ex + ey * ey) / rv - log(2.0 * OR_PI * rv);
            idx[nt++] = k;
        }
        double mx = terms[0];
        for (int k = 1; k < nt; ++k) if (terms[k] > mx) mx = terms[k];
        double s = 0.0;
        for (int k = 0; k < nt; ++k) s += exp(terms[k] - mx);
        for (int k = 1; k < nt; ++k) {
            double rho = exp(terms[k] - mx) / s;
            g[0] += rho * (z[2 * idx[k]] - x[0]) / rv;
            g[1] += rho * (z[2 * idx[k] + 1] - x[1]) / rv;
        }
        break;
    }
    case OR_ARM7:
    case OR_ARM14: { /* zero in the joint velocities of the 14-D model */
        if (!obs_on(mask, 0)) break;
        double org[8][3], zax[8][3];
        arm_frames(m, x, org, zax);
        double e[3];
        for (int c = 0; c < 3; ++c) e[c] = (z[c] - org[7][c]) / p[0];
        for (int i = 0; i < 7; ++i) {
            /* revolute joint i+1 turns about z axis of frame i through origin of frame i */
            double v[3] = { org[7][0] - org[i][0], org[7][1] - org[i][1], org[7][2] - org[i][2] };
            double *za = zax[i];
            double col[3] = { za[1] * v[2] - za[2] * v[1],
                              za[2] * v[0] - za[0] * v[2],
                              za[0] * v[1] - za[1] * v[0] };
            g[i] = col[0] * e[0] + col[1] * e[1] + col[2] * e[2];
        }
        break;
    }
    case OR_SE2: {
        /* gradient of the log of the mixture: responsibilities times the
         * per-landmark gradients; d atan2(dy, dx) = (-dy, dx) / rho^2 */
        if (!obs_on(mask, 0)) break;
        int nl = (int)p[5];
        double terms[8], dx[8], dy[8], rho[8], er[8], eb[8];
        se2_terms(p, z, x, terms, dx, dy, rho, er, eb);
        double mx = terms[0];
        for (int l = 1; l < nl; ++l) if (terms[l] > mx) mx = terms[l];
        double s = 0.0;
        for (int l = 0; l < nl; ++l) s += exp(terms[l] - mx);
        for (int l = 0; l < nl; ++l) {
            if (rho[l] < 1e-12) continue;
            double w = exp(terms[l] - mx) / s;
            double gr = er[l] / p[3] / rho[l], gb = eb[l] / p[4] / (rho[l] * rho[l]);
            g[0] += w * (gr * dx[l] - gb * dy[l]);
            g[1] += w * (gr * dy[l] + gb * dx[l]);
        }
        break;
    }
    case OR_LINGAUSS:
        if (obs_on(mask, 0)) {
            int o = m->obs_dim;
            for (int r = 0; r < o; ++r) {
                double hx = 0.0;
                for (int c = 0; c < d; ++c) hx += p[16 + r * d + c] * x[c];
                double w = (z[r] - hx) / p[32 + r];
                for (int c = 0; c < d; ++c) g[c] += p[16 + r * d + c] * w;
            }
        }
        break;
    }
}

/* ------------------------------------------------------------------------ */
/* Bandwidth: lower median of the squared distances over pairs i < k.        */
/* ------------------------------------------------------------------------ */
static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Threads of the particle loops and the sort (1 = serial). */
void or_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Ascending sort of v[0..M): with several threads, equal chunks are sorted
 * by qsort at once and then merged pairwise, level by level. */
static void sort_doubles(double *v, long M)
{
    int P = or_get_threads();
    if (P <= 1 || M < 4096) {
        qsort(v, (size_t)M, sizeof(double), cmp_double);
        return;
    }
    long chunk = (M + P - 1) / P;
    int nchunks = (int)((M + chunk - 1) / chunk);
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nchunks; ++c) {
        long lo = c * chunk, hi = lo + chunk < M ? lo + chunk : M;
        qsort(v + lo, (size_t)(hi - lo), sizeof(double), cmp_double);
    }
    double *tmp = (double *)malloc(sizeof(double) * (size_t)M);
    double *src = v, *dst = tmp;
    for (long width = chunk; width < M; width *= 2) {
        long pairs = (M + 2 * width - 1) / (2 * width);
#pragma omp parallel for schedule(static)
        for (long q = 0; q < pairs; ++q) {
            long lo = q * 2 * width;
            long mid = lo + width < M ? lo + width : M;
            long hi = lo + 2 * width < M ? lo + 2 * width : M;
            long a = lo, b = mid, o = lo;
            while (a < mid && b < hi) dst[o++] = (src[b] < src[a]) ? src[b++] : src[a++];
            while (a < mid) dst[o++] = src[a++];
            while (b < hi) dst[o++] = src[b++];
        }
        double *t = src; src = dst; dst = t;
    }
    if (src != v) memcpy(v, src, sizeof(double) * (size_t)M);
    free(tmp);
}

/* Sorts v in place and returns element floor((M-1)/2). */
double or_lower_median(double *v, long M)
{
    if (M <= 0) return NAN;
    sort_doubles(v, M);
    return v[(M - 1) / 2];
}

double or_sqdist(const double *a, const double *b, int d)
{
    double s = 0.0;
    for (int c = 0; c < d; ++c) { double r = a[c] - b[c]; s += r * r; }
    return s;
}

/* h = bw_scale * med / ln n; n = 1, a non-positive or a non-finite value
 * give h = 1 (then the single particle's kernel is 1 and its gradient 0). */
double or_bandwidth(const double *x, int n, int d, double bw_scale, double *med_out)
{
    double med = NAN;
    long M = (long)n * (long)(n - 1) / 2;
    if (M > 0) {
        double *v = (double *)malloc(sizeof(double) * (size_t)M);
        /* pair (i, k), i < k, at position i n - i (i + 1) / 2 + k - i - 1 */
#pragma omp parallel for schedule(dynamic, 16)
        for (int i = 0; i < n; ++i) {
            long q = (long)i * n - (long)i * (i + 1) / 2;
            for (int k = i + 1; k < n; ++k) v[q++] = or_sqdist(x + (size_t)i * d, x + (size_t)k * d, d);
        }
        med = or_lower_median(v, M);
        free(v);
    }
    if (med_out) *med_out = med;
    double h = (n > 1) ? bw_scale * med / log((double)n) : NAN;
    if (!(h > 0.0) || !isfinite(h)) h = 1.0;
    return h;
}

/* ------------------------------------------------------------------------ */
/* Scores s_k = grad_x [ log p(z_t | x) + log sum_j w_j N(x; m_j, Q) ] at x_k */
/* (trans_mode 0), or the paper-literal average of transition gradients,     */
/* grad log p(z|x) - Q^-1 (x - mean_j m_j) (trans_mode 1).                   */
/* ------------------------------------------------------------------------ */
void or_scores(const or_model *m, int n_prev, const double *means, const double *log_w,
               const double *z, const uint8_t *mask, int n, const double *x,
               int trans_mode, double *s)
{
    int d = m->d;
    double mean_all[OR_MAXD] = { 0 };
    for (int j = 0; j < n_prev; ++j)
        for (int c = 0; c < d; ++c) mean_all[c] += means[(size_t)j * d + c];
    for (int c = 0; c < d; ++c) mean_all[c] /= (double)n_prev;
#pragma omp parallel
    {
    double *a = (double *)malloc(sizeof(double) * (size_t)(n_prev > 0 ? n_prev : 1));
#pragma omp for schedule(static)
    for (int k = 0; k < n; ++k) {
        const double *xk = x + (size_t)k * d;
        double g[OR_MAXD], mbar[OR_MAXD];
        or_grad_loglik(m, z, mask, xk, g);
        if (trans_mode == 0) {
            double amax = -INFINITY;
            for (int j = 0; j < n_prev; ++j) {
                double lw = log_w ? log_w[j] : -log((double)n_prev);
                a[j] = lw + or_log_transition(m, xk, means + (size_t)j * d);
                if (a[j] > amax) amax = a[j];
            }
            double den = 0.0;
            for (int c = 0; c < d; ++c) mbar[c] = 0.0;
            for (int j = 0; j < n_prev; ++j) {
                double r = exp(a[j] - amax);
                den += r;
                for (int c = 0; c < d; ++c) mbar[c] += r * means[(size_t)j * d + c];
            }
            for (int c = 0; c < d; ++c) mbar[c] /= den;
        } else {
            for (int c = 0; c < d; ++c) mbar[c] = mean_all[c];
        }
        for (int c = 0; c < d; ++c)
            s[(size_t)k * d + c] = g[c] - (xk[c] - mbar[c]) / m->q_var[c];
    }
    free(a);
    }
}

/* Kernels of the Stein direction, functions f(D) of the squared distance
 * D = |x_i - x_k|^2 and the bandwidth h (Sec. V-E compares the three; the
 * paper names them and cites their sources without formulas, so the common
 * forms are taken):
 *   OR_KERNEL_RBF     f = exp(-D / h)                      (Sec. III)
 *   OR_KERNEL_IMQ     f = (1 + D / h)^(-1/2)               inverse multiquadric
 *   OR_KERNEL_MATERN  f = (1 + a) exp(-a), a = sqrt(3 D / h)   Matern, nu = 3/2
 * The gradient with respect to x_k is f'(D) * 2 (x_k - x_i); or_kernel gives
 * f and w = -2 f'(D), so that grad_{x_k} f = w (x_i - x_k):
 *   RBF  w = (2 / h) f;   IMQ  w = (1 / h) f^3;   Matern  w = (3 / h) exp(-a). */
#define OR_KERNEL_RBF 0
#define OR_KERNEL_IMQ 1
#define OR_KERNEL_MATERN 2

void or_kernel(int kernel, double D, double h, double *f, double *w)
{
    if (kernel == OR_KERNEL_IMQ) {
        double v = 1.0 / sqrt(1.0 + D / h);
        *f = v;
        *w = v * v * v / h;
    } else if (kernel == OR_KERNEL_MATERN) {
        double a = sqrt(3.0 * D / h);
        double e = exp(-a);
        *f = (1.0 + a) * e;
        *w = 3.0 * e / h;
    } else {
        double v = exp(-D / h);
        *f = v;
        *w = 2.0 * v / h;
    }
}

/* phi_i = (1/n) sum_k [ kappa_ik s_k + grad_{x_k} kappa_ik ],
 * kappa_ik = f(|x_i - x_k|^2), grad_{x_k} kappa_ik = w_ik (x_i - x_k). */
void or_stein_phi(int n, int d, const double *x, const double *s, double h, int kernel, double *phi)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        const double *xi = x + (size_t)i * d;
        double acc[OR_MAXD] = { 0 };
        for (int k = 0; k < n; ++k) {
            const double *xk = x + (size_t)k * d;
            double kap, w;
            or_kernel(kernel, or_sqdist(xi, xk, d), h, &kap, &w);
            for (int c = 0; c < d; ++c)
                acc[c] += kap * s[(size_t)k * d + c] + w * (xi[c] - xk[c]);
        }
        for (int c = 0; c < d; ++c) phi[(size_t)i * d + c] = acc[c] / (double)n;
    }
}

static int all_finite(const double *v, size_t cnt)
{
    for (size_t q = 0; q < cnt; ++q) if (!isfinite(v[q])) return 0;
    return 1;
}

/* One time step of SVGD (Algorithm 2 steps 1 / 2).  x [n,d] holds the initial
 * particles on entry and the updated ones on exit.  Every quantity of
 * iteration l is read from the iteration-l particles (all particles move
 * together).  h_out [n_iter] receives the bandwidth of each iteration. */
int or_svgd_step(const or_model *m, int t, int n_prev, const double *x_prev, const double *log_w,
                 const double *z, const uint8_t *mask, int n, double *x,
                 int n_iter, double step, double bw_scale, int bw_mode, int trans_mode,
                 int kernel, double *h_out)
{
    if (n <= 0 || n_prev <= 0 || n_iter < 0) return OR_INVALID;
    int d = m->d;
    size_t nd = (size_t)n * d;
    double *means = (double *)malloc(sizeof(double) * (size_t)n_prev * d);
    double *s = (double *)malloc(sizeof(double) * nd);
    double *phi = (double *)malloc(sizeof(double) * nd);
    for (int j = 0; j < n_prev; ++j)
        or_transition_mean(m, t, x_prev + (size_t)j * d, means + (size_t)j * d);
    double h = 1.0;
    for (int l = 0; l < n_iter; ++l) {
        if (bw_mode == 0 || l == 0) h = or_bandwidth(x, n, d, bw_scale, NULL);
        if (h_out) h_out[l] = h;
        or_scores(m, n_prev, means, log_w, z, mask, n, x, trans_mode, s);
        or_stein_phi(n, d, x, s, h, kernel, phi);
        for (size_t q = 0; q < nd; ++q) x[q] += step * phi[q];
    }
    free(means); free(s); free(phi);
    return all_finite(x, nd) ? OR_OK : OR_NONFINITE;
}

/* ------------------------------------------------------------------------ */
/* Forward recursion (eq. forward_recursion).  c_ij = A_ij + phi_prev(j);    */
/* psi(i) = lowest j attaining max_j c_ij; phi(i) = c_{i psi(i)} + ell_i.    */
/* flags(i) = 1 when the best value among j != psi(i) is within              */
/* tie_tol * max(1, |best|) of the best.                                      */
/* ------------------------------------------------------------------------ */
static int forward_row(int n_prev, const double *c, double ell, double tie_tol,
                       double *phi_i, int32_t *psi_i, uint8_t *flag_i)
{
    int bad = 0;
    int arg = 0;
    double best = c[0];
    if (isnan(c[0])) bad = 1;
    for (int j = 1; j < n_prev; ++j) {
        if (isnan(c[j])) bad = 1;
        if (c[j] > best) { best = c[j]; arg = j; }
    }
    double second = -INFINITY;
    for (int j = 0; j < n_prev; ++j)
        if (j != arg && c[j] > second) second = c[j];
    *psi_i = arg;
    *phi_i = best + ell;
    if (flag_i) {
        double scale = fabs(best) > 1.0 ? fabs(best) : 1.0;
        *flag_i = (uint8_t)(n_prev > 1 && second >= best - tie_tol * scale);
    }
    if (isnan(ell) || isnan(*phi_i)) bad = 1;
    return bad;
}

int or_viterbi_lattice(int n, int n_prev, const double *A, const double *ell, const double *phi_prev,
                       double tie_tol, double *phi, int32_t *psi, uint8_t *flags)
{
    if (n <= 0 || n_prev <= 0) return OR_INVALID;
    double *c = (double *)malloc(sizeof(double) * (size_t)n_prev);
    int bad = 0;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n_prev; ++j) c[j] = A[(size_t)i * n_prev + j] + phi_prev[j];
        bad |= forward_row(n_prev, c, ell[i], tie_tol, phi + i, psi + i, flags ? flags + i : NULL);
    }
    free(c);
    return bad ? OR_NONFINITE : OR_OK;
}

/* Particle mode: A_ij = log N(x_t^i; f_t(x_{t-1}^j), Q), ell_i = log p(z_t | x_t^i). */
int or_viterbi_particle(const or_model *m, int t, int n_prev, const double *x_prev,
                        const double *phi_prev, const double *z, const uint8_t *mask,
                        int n, const double *x, double tie_tol,
                        double *phi, int32_t *psi, uint8_t *flags)
{
    if (n <= 0 || n_prev <= 0) return OR_INVALID;
    int d = m->d;
    double *means = (double *)malloc(sizeof(double) * (size_t)n_prev * d);
    for (int j = 0; j < n_prev; ++j)
        or_transition_mean(m, t, x_prev + (size_t)j * d, means + (size_t)j * d);
    int bad = 0;
#pragma omp parallel reduction(|:bad)
    {
    double *c = (double *)malloc(sizeof(double) * (size_t)n_prev);
#pragma omp for schedule(static)
    for (int i = 0; i < n; ++i) {
        const double *xi = x + (size_t)i * d;
        for (int j = 0; j < n_prev; ++j)
            c[j] = or_log_transition(m, xi, means + (size_t)j * d) + phi_prev[j];
        double ell = or_loglik(m, z, mask, xi);
        bad |= forward_row(n_prev, c, ell, tie_tol, phi + i, psi + i, flags ? flags + i : NULL);
    }
    free(c);
    }
    free(means);
    return bad ? OR_NONFINITE : OR_OK;
}

/* The log-transition lattice and log-likelihoods of particle mode, for
 * feeding lattice mode. */
void or_particle_lattice(const or_model *m, int t, int n_prev, const double *x_prev,
                         const double *z, const uint8_t *mask, int n, const double *x,
                         double *A, double *ell)
{
    int d = m->d;
    double mean[OR_MAXD];
    for (int j = 0; j < n_prev; ++j) {
        or_transition_mean(m, t, x_prev + (size_t)j * d, mean);
        for (int i = 0; i < n; ++i)
            A[(size_t)i * n_prev + j] = or_log_transition(m, x + (size_t)i * d, mean);
    }
    for (int i = 0; i < n; ++i) ell[i] = or_loglik(m, z, mask, x + (size_t)i * d);
}

/* Backtracking: i_T = lowest argmax phi_T; i_{t-1} = psi_t(i_t).  psi is
 * [T, n] with row t-1 holding step t.  idx_out [T] (entry t-1 = i_t). */
int or_backtrack(int T, int n, const int32_t *psi, const double *phi_T, int32_t *idx_out, double *J)
{
    if (T <= 0 || n <= 0) return OR_INVALID;
    int arg = 0;
    for (int i = 1; i < n; ++i) if (phi_T[i] > phi_T[arg]) arg = i;
    idx_out[T - 1] = arg;
    for (int t = T; t >= 2; --t) {
        int32_t prev = psi[(size_t)(t - 1) * n + idx_out[t - 1]];
        if (prev < 0 || prev >= n) return OR_INVALID;
        idx_out[t - 2] = prev;
    }
    *J = phi_T[arg];
    return isfinite(*J) ? OR_OK : OR_NONFINITE;
}

/* J(s) = sum_t [ log p(s_t | s_{t-1}) + log p(z_t | s_t) ] (Theorem IV.1, the
 * constant log p(s_0) of the sharp prior left out), accumulated in the same
 * order as the forward recursion: J_t = (A_t + J_{t-1}) + ell_t.
 * path [T+1, d] with path[0] = x_0. */
double or_path_score(const or_model *m, int T, const double *path, const double *z,
                     const uint8_t *mask)
{
    int d = m->d;
    double J = 0.0, mean[OR_MAXD];
    for (int t = 1; t <= T; ++t) {
        or_transition_mean(m, t, path + (size_t)(t - 1) * d, mean);
        double A = or_log_transition(m, path + (size_t)t * d, mean);
        double ell = or_loglik(m, z + (size_t)(t - 1) * m->obs_dim,
                               mask ? mask + (size_t)(t - 1) * m->n_obs : NULL, path + (size_t)t * d);
        J = (A + J) + ell;
    }
    return J;
}

/* Predictive initial particles: x_i = f_t(x_prev[i mod n_prev]) + sqrt(q) * xi_{t,i}. */
void or_predictive_init(const or_model *m, int t, int n_prev, const double *x_prev, int n,
                        uint64_t seed, uint32_t seq, double *x)
{
    int d = m->d;
    double mean[OR_MAXD], nz[OR_MAXD];
    for (int i = 0; i < n; ++i) {
        or_transition_mean(m, t, x_prev + (size_t)(i % n_prev) * d, mean);
        or_normals(seed, seq, (uint32_t)t, (uint32_t)i, d, nz);
        for (int c = 0; c < d; ++c) x[(size_t)i * d + c] = mean[c] + sqrt(m->q_var[c]) * nz[c];
    }
}

/* Algorithm 2 end to end for one sequence.  z [T, obs_dim], mask [T, n_obs]
 * or NULL.  Outputs: xmap [T+1, d], J, and optionally every step's particles
 * [T, n, d] and forward-recursion tables phi [T, n], psi [T, n]. */
int or_run_sequence(const or_model *m, int T, int n, const double *x0, const double *z,
                    const uint8_t *mask, uint64_t seed, uint32_t seq,
                    int n_iter, double step, double bw_scale, int bw_mode, int trans_mode,
                    int kernel, int weights, double *xmap, double *J, double *particles_out, double *phi_out,
                    int32_t *psi_out, int32_t *idx_out)
{
    if (T <= 0 || n <= 0) return OR_INVALID;
    int d = m->d, status = OR_OK;
    size_t nd = (size_t)n * d;
    double *parts = (double *)malloc(sizeof(double) * nd * (size_t)T);
    int32_t *psi = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * T);
    double *phi = (double *)malloc(sizeof(double) * (size_t)n * T);
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)T);
    double zero = 0.0;
    for (int t = 1; t <= T; ++t) {
        const double *xprev = (t == 1) ? x0 : parts + nd * (size_t)(t - 2);
        const double *phiprev = (t == 1) ? &zero : phi + (size_t)n * (t - 2);
        int n_prev = (t == 1) ? 1 : n;
        const double *zt = z + (size_t)(t - 1) * m->obs_dim;
        const uint8_t *mt = mask ? mask + (size_t)(t - 1) * m->n_obs : NULL;
        double *xt = parts + nd * (size_t)(t - 1);
        or_predictive_init(m, t, n_prev, xprev, n, seed, seq, xt);
        const double *lw = (weights == 1 && t > 1) ? phiprev : NULL;
        int st = or_svgd_step(m, t, n_prev, xprev, lw, zt, mt, n, xt, n_iter, step, bw_scale,
                              bw_mode, trans_mode, kernel, NULL);
        if (st != OR_OK) status = st;
        st = or_viterbi_particle(m, t, n_prev, xprev, phiprev, zt, mt, n, xt, 0.0,
                                 phi + (size_t)n * (t - 1), psi + (size_t)n * (t - 1), NULL);
        if (st != OR_OK) status = st;
    }
    int st = or_backtrack(T, n, psi, phi + (size_t)n * (T - 1), idx, J);
    if (st != OR_OK && status == OR_OK) status = st;
    for (int c = 0; c < d; ++c) xmap[c] = x0[c];
    for (int t = 1; t <= T; ++t)
        for (int c = 0; c < d; ++c)
            xmap[(size_t)t * d + c] = parts[nd * (size_t)(t - 1) + (size_t)idx[t - 1] * d + c];
    if (particles_out) memcpy(particles_out, parts, sizeof(double) * nd * (size_t)T);
    if (phi_out) memcpy(phi_out, phi, sizeof(double) * (size_t)n * T);
    if (psi_out) memcpy(psi_out, psi, sizeof(int32_t) * (size_t)n * T);
    if (idx_out) memcpy(idx_out, idx, sizeof(int32_t) * (size_t)T);
    free(parts); free(psi); free(phi); free(idx);
    return status;
}
