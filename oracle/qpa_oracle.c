/*
 * qpa_oracle.c -- plain, slow CPU oracle for replica-batched Parallel Annealing (PA).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library or its Python binding
 * links, loads or calls this file; only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg do.  It shares no code, header, table or constant
 * generator with the HIP path.
 *
 * What it computes (paper: "VeloxQ: A Fast and Efficient QUBO Solver", arXiv 2501.19221):
 *   - QUBO objective E(x) = x^T Q x + c^T x over x in {0,1}^n with symmetric Q
 *     (Sec. II, eq. (1), written in the symmetric-matrix form), and the Ising objective
 *     H(s) = sum_{i<j} J_ij s_i s_j + sum_i b_i s_i over s in {-1,+1}^n (Sec. II, eq. (2);
 *     matrix form (1/2) s^T J s + s^T b of App. C).
 *   - The QUBO -> Ising map obtained from x = (1+s)/2 (App. A).  With a symmetric Q the
 *     exact identity is 2 E(x) = H(s) + K with J = Q with its diagonal removed,
 *     b = Q 1 + c and K = (1/2) 1^T Q 1 + (1/2) tr Q + 1^T c.  (The additive constants
 *     printed in App. A carry the opposite sign; the reading used here is the one that
 *     exhaustive enumeration confirms -- see the tests.)
 *   - Parallel Annealing dynamics (App. B): analog spins x in [-1,1], binarised spins
 *     s = sign(x) (sign(0) read as +1), gradient lambda(t) x + J s + b evaluated with the
 *     target part on binarised spins, heavy-ball momentum m <- alpha m - eta grad,
 *     position update x <- x + m, then clipping of x to [-1,1].  All variables of a
 *     replica are updated synchronously from the state of the previous step.
 *   - The relaxed variant used for gradients (analog spins used in the target part,
 *     s := x) and its reverse-mode adjoint with respect to eta, alpha and every
 *     lambda_t, derived by hand from the same update rule.
 *   - Exhaustive ground-state search for small n (Sec. VII.A uses brute force as the
 *     exact reference).
 *   - The adiabatic Simulated Bifurcation Machine (App. B, Hamilton's equations of the
 *     oscillator network) integrated with symplectic Euler, on the same (J, b).
 *
 * Arithmetic contract of the dynamics: FP32, every operation rounded separately in the
 * order written (this file is compiled with -ffp-contract=off), integer couplings summed
 * exactly in int64 and then converted, float couplings summed in FP32 in ascending
 * column order.  Energies are exact in int64 for integer instances, FP64 otherwise.
 * The FP64 relaxed forward/adjoint is plain double arithmetic; its FP32 variant rounds
 * the state, the adjoint vectors and the products (one fused multiply-add per term, in
 * ascending column order) to single precision.
 *
 * Parity pins live in tests/ (brute force vs naive enumeration, App. A identities,
 * closed forms of the update, planted optima, finite differences for the adjoint,
 * SplitMix64 reference vectors; for SBM a hand-worked two-spin fixture, first-order
 * convergence to a library ODE solution, bounded energy error, sign conventions).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ------------------------------------------------------------------------------------
 * Counter-based draw: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014).  The generator's state advances by the golden-ratio
 * increment and each output is the state passed through the 64-bit finaliser; the k-th
 * output (k >= 1) of a generator seeded with `seed` is therefore mix(seed + k*gamma).
 * ---------------------------------------------------------------------------------- */
static uint64_t sm64_finalise(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t orc_sm64_output(uint64_t seed, uint64_t k)
{
    return sm64_finalise(seed + k * 0x9e3779b97f4a7c15ULL);
}

/* Initial analog spins (the paper leaves the initial state open): replica r, variable i
 * draws the (r*n + i + 1)-th SplitMix64 output, keeps its top 24 bits as u in [0,1) on an
 * exact 2^-24 grid, and sets x0 = sigma0 * (2u - 1); momentum starts at zero.
 * r0 is the global index of the first replica written, so any replica subset is
 * reproducible on its own. */
void orc_pa_init(int64_t n, int64_t r0, int64_t nrep, uint64_t seed, float sigma0,
                 float *x, float *m)
{
    for (int64_t r = 0; r < nrep; ++r) {
        for (int64_t i = 0; i < n; ++i) {
            uint64_t k = (uint64_t)((r0 + r) * n + i) + 1u;
            uint64_t top = orc_sm64_output(seed, k) >> 40;          /* 24 bits */
            float u = (float)top * (1.0f / 16777216.0f);             /* exact */
            float v = 2.0f * u;                                       /* exact */
            v = v - 1.0f;                                             /* exact */
            x[r * n + i] = sigma0 * v;
            m[r * n + i] = 0.0f;
        }
    }
}

/* Linear annealing schedule: lambda(t) falls from lambda0 to zero over T steps
 * (App. B only asks for a gradual decrease from a large value to zero). */
void orc_lambda_linear(int64_t T, float lambda0, float *lam)
{
    for (int64_t t = 0; t < T; ++t) {
        float frac = (float)t / (float)T;
        float one_minus = 1.0f - frac;
        lam[t] = lambda0 * one_minus;
    }
}

/* ------------------------------------------------------------------------------------
 * App. A: QUBO (symmetric Q, linear c) -> Ising (J, b) with 2E(x) = H(s) + K.
 * ---------------------------------------------------------------------------------- */
void orc_qubo_to_ising_i64(int64_t n, const int32_t *Q, const int64_t *c,
                           int32_t *J, int64_t *b, int64_t *K)
{
    int64_t total = 0, trace = 0, lin = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t row = 0;
        for (int64_t j = 0; j < n; ++j) {
            int32_t q = Q[i * n + j];
            row += q;
            J[i * n + j] = (i == j) ? 0 : q;
        }
        b[i] = row + c[i];
        total += row;
        trace += Q[i * n + i];
        lin += c[i];
    }
    /* (1/2)(1^T Q 1 + tr Q) = sum_{i<j} Q_ij + tr Q is an integer for symmetric Q */
    *K = (total + trace) / 2 + lin;
}

void orc_qubo_to_ising_f64(int64_t n, const double *Q, const double *c,
                           double *J, double *b, double *K)
{
    double total = 0.0, trace = 0.0, lin = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double row = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double q = Q[i * n + j];
            row += q;
            J[i * n + j] = (i == j) ? 0.0 : q;
        }
        b[i] = row + c[i];
        total += row;
        trace += Q[i * n + i];
        lin += c[i];
    }
    *K = 0.5 * total + 0.5 * trace + lin;
}

/* ------------------------------------------------------------------------------------
 * Energies.  Ising: eq. (2) summed over i<j as written; QUBO: x^T Q x + c^T x.
 * ---------------------------------------------------------------------------------- */
int64_t orc_ising_energy_i64(int64_t n, const int32_t *J, const int64_t *b, const int8_t *s)
{
    int64_t e = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j)
            e += (int64_t)J[i * n + j] * s[i] * s[j];
        e += b[i] * s[i];
    }
    return e;
}

double orc_ising_energy_f64(int64_t n, const double *J, const double *b, const int8_t *s)
{
    double e = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j)
            e += J[i * n + j] * (double)(s[i] * s[j]);
        e += b[i] * (double)s[i];
    }
    return e;
}

int64_t orc_qubo_energy_i64(int64_t n, const int32_t *Q, const int64_t *c, const int8_t *x)
{
    int64_t e = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!x[i]) continue;
        for (int64_t j = 0; j < n; ++j)
            if (x[j]) e += Q[i * n + j];
        e += c[i];
    }
    return e;
}

double orc_qubo_energy_f64(int64_t n, const double *Q, const double *c, const int8_t *x)
{
    double e = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!x[i]) continue;
        for (int64_t j = 0; j < n; ++j)
            if (x[j]) e += Q[i * n + j];
        e += c[i];
    }
    return e;
}

/* Sparse Ising energy: every stored entry (i,j) with j>i is counted once, so a symmetric
 * CSR gives eq. (2) exactly. */
int64_t orc_ising_energy_csr_i64(int64_t n, const int64_t *rp, const int32_t *col,
                                 const int32_t *w, const int64_t *b, const int8_t *s)
{
    int64_t e = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            int64_t j = col[k];
            if (j > i) e += (int64_t)w[k] * s[i] * s[j];
        }
        e += b[i] * s[i];
    }
    return e;
}

double orc_ising_energy_csr_f64(int64_t n, const int64_t *rp, const int32_t *col,
                                const double *w, const double *b, const int8_t *s)
{
    double e = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            int64_t j = col[k];
            if (j > i) e += w[k] * (double)(s[i] * s[j]);
        }
        e += b[i] * (double)s[i];
    }
    return e;
}

/* ------------------------------------------------------------------------------------
 * Exhaustive search (Sec. VII.A): walk all 2^n spin states in Gray-code order, keeping
 * every local field J s + b up to date after each single flip, so that the energy change
 * of flipping spin k is -2 s_k f_k.  Returns the minimum of H; best_s receives the first
 * minimiser met in Gray order (starting from all spins -1).
 * ---------------------------------------------------------------------------------- */
int64_t orc_bruteforce_ising_i64(int64_t n, const int32_t *J, const int64_t *b, int8_t *best_s)
{
    int8_t *s = (int8_t *)malloc((size_t)n);
    int64_t *f = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) s[i] = -1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t acc = b[i];
        for (int64_t j = 0; j < n; ++j) acc += (int64_t)J[i * n + j] * s[j];
        f[i] = acc;
    }
    int64_t e = orc_ising_energy_i64(n, J, b, s);
    int64_t best = e;
    memcpy(best_s, s, (size_t)n);
    uint64_t count = 1ull << n;
    for (uint64_t g = 1; g < count; ++g) {
        int64_t k = __builtin_ctzll(g);                 /* bit that changes in Gray order */
        e += -2 * (int64_t)s[k] * f[k];                 /* J has a zero diagonal */
        int8_t old = s[k];
        s[k] = (int8_t)(-old);
        for (int64_t i = 0; i < n; ++i)
            f[i] += (int64_t)J[i * n + k] * (s[k] - old);
        if (e < best) {
            best = e;
            memcpy(best_s, s, (size_t)n);
        }
    }
    free(s);
    free(f);
    return best;
}

/* ------------------------------------------------------------------------------------
 * PA steps (App. B).  x, m are [nrep][n] row-major FP32 and are advanced in place from
 * step t0 up to (not including) t1 with lambda table lam[t].  If h_out is given it
 * receives the local fields J s + b of the last step taken.
 * ---------------------------------------------------------------------------------- */
static void pa_update_row(int64_t n, const float *h, float lam, float eta, float alpha,
                          float *x, float *m)
{
    for (int64_t i = 0; i < n; ++i) {
        float p = lam * x[i];
        float g = p + h[i];                 /* gradient: lambda x + (J s + b) */
        float am = alpha * m[i];
        float eg = eta * g;
        float mn = am - eg;                 /* m <- alpha m - eta grad */
        float y = x[i] + mn;                /* x <- x + m */
        if (y > 1.0f) y = 1.0f;             /* clip to [-1, 1] */
        if (y < -1.0f) y = -1.0f;
        m[i] = mn;
        x[i] = y;
    }
}

/* The update alone, for `count` (variable, replica) pairs given their fields h. */
void orc_pa_update_f32(int64_t count, const float *h, float lam, float eta, float alpha,
                       float *x, float *m)
{
    pa_update_row(count, h, lam, eta, alpha, x, m);
}

void orc_pa_steps_dense_i64(int64_t n, const int32_t *J, const int64_t *b, int64_t nrep,
                            float *x, float *m, int64_t t0, int64_t t1, const float *lam,
                            float eta, float alpha, float *h_out)
{
    int8_t *s = (int8_t *)malloc((size_t)n);
    float *h = (float *)malloc(sizeof(float) * (size_t)n);
    for (int64_t r = 0; r < nrep; ++r) {
        float *xr = x + r * n, *mr = m + r * n;
        for (int64_t t = t0; t < t1; ++t) {
            for (int64_t j = 0; j < n; ++j) s[j] = (xr[j] >= 0.0f) ? 1 : -1;
            for (int64_t i = 0; i < n; ++i) {
                int64_t acc = 0;
                for (int64_t j = 0; j < n; ++j) acc += (int64_t)J[i * n + j] * s[j];
                h[i] = (float)(acc + b[i]);
            }
            pa_update_row(n, h, lam[t], eta, alpha, xr, mr);
        }
        if (h_out && t1 > t0) memcpy(h_out + r * n, h, sizeof(float) * (size_t)n);
    }
    free(s);
    free(h);
}

void orc_pa_steps_dense_f32(int64_t n, const float *J, const float *b, int64_t nrep,
                            float *x, float *m, int64_t t0, int64_t t1, const float *lam,
                            float eta, float alpha, float *h_out)
{
    float *s = (float *)malloc(sizeof(float) * (size_t)n);
    float *h = (float *)malloc(sizeof(float) * (size_t)n);
    for (int64_t r = 0; r < nrep; ++r) {
        float *xr = x + r * n, *mr = m + r * n;
        for (int64_t t = t0; t < t1; ++t) {
            for (int64_t j = 0; j < n; ++j) s[j] = (xr[j] >= 0.0f) ? 1.0f : -1.0f;
            for (int64_t i = 0; i < n; ++i) {
                float acc = 0.0f;
                for (int64_t j = 0; j < n; ++j) acc += J[i * n + j] * s[j];
                h[i] = acc + b[i];
            }
            pa_update_row(n, h, lam[t], eta, alpha, xr, mr);
        }
        if (h_out && t1 > t0) memcpy(h_out + r * n, h, sizeof(float) * (size_t)n);
    }
    free(s);
    free(h);
}

void orc_pa_steps_csr_i64(int64_t n, const int64_t *rp, const int32_t *col, const int32_t *w,
                          const int64_t *b, int64_t nrep, float *x, float *m, int64_t t0,
                          int64_t t1, const float *lam, float eta, float alpha, float *h_out)
{
    int8_t *s = (int8_t *)malloc((size_t)n);
    float *h = (float *)malloc(sizeof(float) * (size_t)n);
    for (int64_t r = 0; r < nrep; ++r) {
        float *xr = x + r * n, *mr = m + r * n;
        for (int64_t t = t0; t < t1; ++t) {
            for (int64_t j = 0; j < n; ++j) s[j] = (xr[j] >= 0.0f) ? 1 : -1;
            for (int64_t i = 0; i < n; ++i) {
                int64_t acc = 0;
                for (int64_t k = rp[i]; k < rp[i + 1]; ++k) acc += (int64_t)w[k] * s[col[k]];
                h[i] = (float)(acc + b[i]);
            }
            pa_update_row(n, h, lam[t], eta, alpha, xr, mr);
        }
        if (h_out && t1 > t0) memcpy(h_out + r * n, h, sizeof(float) * (size_t)n);
    }
    free(s);
    free(h);
}

void orc_pa_steps_csr_f32(int64_t n, const int64_t *rp, const int32_t *col, const float *w,
                          const float *b, int64_t nrep, float *x, float *m, int64_t t0,
                          int64_t t1, const float *lam, float eta, float alpha, float *h_out)
{
    float *s = (float *)malloc(sizeof(float) * (size_t)n);
    float *h = (float *)malloc(sizeof(float) * (size_t)n);
    for (int64_t r = 0; r < nrep; ++r) {
        float *xr = x + r * n, *mr = m + r * n;
        for (int64_t t = t0; t < t1; ++t) {
            for (int64_t j = 0; j < n; ++j) s[j] = (xr[j] >= 0.0f) ? 1.0f : -1.0f;
            for (int64_t i = 0; i < n; ++i) {
                float acc = 0.0f;
                for (int64_t k = rp[i]; k < rp[i + 1]; ++k) acc += w[k] * s[col[k]];
                h[i] = acc + b[i];
            }
            pa_update_row(n, h, lam[t], eta, alpha, xr, mr);
        }
        if (h_out && t1 > t0) memcpy(h_out + r * n, h, sizeof(float) * (size_t)n);
    }
    free(s);
    free(h);
}

/* One PA step restricted to the listed rows, from a full state (x, m) of one replica:
 * writes the field, new x and new m of each listed row.  Used to check single outputs of
 * a very large instance one by one. */
void orc_pa_step_rows_csr_i64(int64_t n, const int64_t *rp, const int32_t *col, const int32_t *w,
                              const int64_t *b, const float *x, const float *m, int64_t nrows,
                              const int64_t *rows, float lam, float eta, float alpha,
                              float *h_out, float *x_out, float *m_out)
{
    (void)n;
    for (int64_t q = 0; q < nrows; ++q) {
        int64_t i = rows[q];
        int64_t acc = 0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            int64_t j = col[k];
            acc += (int64_t)w[k] * ((x[j] >= 0.0f) ? 1 : -1);
        }
        float h = (float)(acc + b[i]);
        float xi = x[i], mi = m[i];
        pa_update_row(1, &h, lam, eta, alpha, &xi, &mi);
        h_out[q] = h;
        x_out[q] = xi;
        m_out[q] = mi;
    }
}

/* ------------------------------------------------------------------------------------
 * BF16 storage of float couplings: round-to-nearest-even of J / 2^e to 8 significant
 * bits, with e the smallest integer such that max|J| <= 2^e.  The returned array holds
 * 2^e * bf16(J / 2^e) as FP32 (exact), i.e. the couplings the BF16 field sees.
 * ---------------------------------------------------------------------------------- */
static float bf16_round_nearest_even(float v)
{
    uint32_t u;
    memcpy(&u, &v, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return v;       /* inf / nan untouched */
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

int32_t orc_bf16_scale_exponent(int64_t count, const float *J)
{
    float mx = 0.0f;
    for (int64_t k = 0; k < count; ++k) {
        float a = fabsf(J[k]);
        if (a > mx) mx = a;
    }
    if (mx == 0.0f) return 0;
    int e;
    float f = frexpf(mx, &e);      /* mx = f * 2^e, f in [0.5, 1) */
    if (f == 0.5f) e -= 1;         /* exact power of two: mx = 2^(e-1) */
    return (int32_t)e;
}

void orc_bf16_quantise(int64_t count, const float *J, int32_t e, float *Jq)
{
    for (int64_t k = 0; k < count; ++k) {
        float scaled = ldexpf(J[k], -e);
        Jq[k] = ldexpf(bf16_round_nearest_even(scaled), e);
    }
}

/* ------------------------------------------------------------------------------------
 * Relaxed PA (s := x) in FP64 and its reverse-mode adjoint.
 * Loss: L = (1/nrep) sum_r [ (1/2) x_T^T J x_T + b^T x_T ] over the replicas given.
 * Forward step t: g = lam_t x + J x + b; m' = alpha m - eta g; y = x + m'; x' = clip(y).
 * Reverse (mu_{T+1} = 0, xbar_T = dL/dx_T):
 *   ybar = xbar_{t+1} * [ |y_{t+1}| <= 1 ]
 *   mu   = ybar + alpha * mu_next                 (total derivative w.r.t. m_{t+1})
 *   dL/deta     += <mu, -g_t>
 *   dL/dalpha   += <mu, m_t>
 *   dL/dlam_t    = <mu, -eta x_t>
 *   xbar_t = ybar - eta (lam_t mu + J mu)
 * The dense variant is below; the whole trajectory is stored (no checkpointing).
 * ---------------------------------------------------------------------------------- */
static void matvec_dense_f64(int64_t n, const double *J, const double *v, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j) acc += J[i * n + j] * v[j];
        out[i] = acc;
    }
}

static void matvec_csr_f64(int64_t n, const int64_t *rp, const int32_t *col, const double *w,
                           const double *v, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) acc += w[k] * v[col[k]];
        out[i] = acc;
    }
}

/* fmt 0: dense J (n*n); fmt 1: CSR (rp, col, w). */
static void matvec_any(int fmt, int64_t n, const double *J, const int64_t *rp,
                       const int32_t *col, const double *w, const double *v, double *out)
{
    if (fmt == 0) matvec_dense_f64(n, J, v, out);
    else matvec_csr_f64(n, rp, col, w, v, out);
}

static double relaxed_grad(int fmt, int64_t n, const double *J, const int64_t *rp,
                           const int32_t *col, const double *w, const double *b, int64_t nrep,
                           const double *x0, const double *m0, int64_t T, const double *lam,
                           double eta, double alpha, double norm, double *d_eta,
                           double *d_alpha, double *d_lam, double *xT)
{
    double *X = (double *)malloc(sizeof(double) * (size_t)((T + 1) * n));
    double *M = (double *)malloc(sizeof(double) * (size_t)((T + 1) * n));
    double *Y = (double *)malloc(sizeof(double) * (size_t)((T + 1) * n));
    double *G = (double *)malloc(sizeof(double) * (size_t)(T * n));
    double *f = (double *)malloc(sizeof(double) * (size_t)n);
    double *xbar = (double *)malloc(sizeof(double) * (size_t)n);
    double *mu = (double *)malloc(sizeof(double) * (size_t)n);
    double *ybar = (double *)malloc(sizeof(double) * (size_t)n);
    double loss = 0.0;
    if (d_eta) *d_eta = 0.0;
    if (d_alpha) *d_alpha = 0.0;
    if (d_lam) for (int64_t t = 0; t < T; ++t) d_lam[t] = 0.0;

    for (int64_t r = 0; r < nrep; ++r) {
        memcpy(X, x0 + r * n, sizeof(double) * (size_t)n);
        if (m0) memcpy(M, m0 + r * n, sizeof(double) * (size_t)n);
        else memset(M, 0, sizeof(double) * (size_t)n);
        for (int64_t t = 0; t < T; ++t) {
            const double *x = X + t * n, *mm = M + t * n;
            double *xn = X + (t + 1) * n, *mn = M + (t + 1) * n, *yn = Y + (t + 1) * n;
            double *g = G + t * n;
            matvec_any(fmt, n, J, rp, col, w, x, f);
            for (int64_t i = 0; i < n; ++i) {
                g[i] = lam[t] * x[i] + f[i] + b[i];
                mn[i] = alpha * mm[i] - eta * g[i];
                yn[i] = x[i] + mn[i];
                xn[i] = yn[i] > 1.0 ? 1.0 : (yn[i] < -1.0 ? -1.0 : yn[i]);
            }
        }
        const double *xt = X + T * n;
        if (xT) memcpy(xT + r * n, xt, sizeof(double) * (size_t)n);
        matvec_any(fmt, n, J, rp, col, w, xt, f);
        double e = 0.0;
        for (int64_t i = 0; i < n; ++i) e += 0.5 * xt[i] * f[i] + b[i] * xt[i];
        loss += e * norm;
        if (!(d_eta || d_alpha || d_lam)) continue;
        for (int64_t i = 0; i < n; ++i) {
            xbar[i] = (f[i] + b[i]) * norm;
            mu[i] = 0.0;
        }
        for (int64_t t = T - 1; t >= 0; --t) {
            const double *x = X + t * n, *mm = M + t * n, *yn = Y + (t + 1) * n;
            const double *g = G + t * n;
            double se = 0.0, sa = 0.0, sl = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                ybar[i] = (fabs(yn[i]) <= 1.0) ? xbar[i] : 0.0;
                mu[i] = ybar[i] + alpha * mu[i];
                se += mu[i] * (-g[i]);
                sa += mu[i] * mm[i];
                sl += mu[i] * (-eta * x[i]);
            }
            if (d_eta) *d_eta += se;
            if (d_alpha) *d_alpha += sa;
            if (d_lam) d_lam[t] += sl;
            matvec_any(fmt, n, J, rp, col, w, mu, f);
            for (int64_t i = 0; i < n; ++i)
                xbar[i] = ybar[i] - eta * (lam[t] * mu[i] + f[i]);
        }
    }
    free(X); free(M); free(Y); free(G); free(f); free(xbar); free(mu); free(ybar);
    return loss;
}

/* Returns L; gradient pointers may be NULL (forward only).  x0 is [nrep][n]; m0 may be
 * NULL for a zero initial momentum.  norm is the 1/(replica count) factor of the mean
 * (passed in so that a subset can contribute its share of a larger mean). */
double orc_relaxed_grad_dense_f64(int64_t n, const double *J, const double *b, int64_t nrep,
                                  const double *x0, const double *m0, int64_t T,
                                  const double *lam, double eta, double alpha, double norm,
                                  double *d_eta, double *d_alpha, double *d_lam, double *xT)
{
    return relaxed_grad(0, n, J, NULL, NULL, NULL, b, nrep, x0, m0, T, lam, eta, alpha, norm,
                        d_eta, d_alpha, d_lam, xT);
}

double orc_relaxed_grad_csr_f64(int64_t n, const int64_t *rp, const int32_t *col,
                                const double *w, const double *b, int64_t nrep,
                                const double *x0, const double *m0, int64_t T,
                                const double *lam, double eta, double alpha, double norm,
                                double *d_eta, double *d_alpha, double *d_lam, double *xT)
{
    return relaxed_grad(1, n, NULL, rp, col, w, b, nrep, x0, m0, T, lam, eta, alpha, norm,
                        d_eta, d_alpha, d_lam, xT);
}

/* The same relaxed forward pass and adjoint in single precision: state x, m, the
 * adjoint vectors xbar, mu and the products J v in FP32, every operation rounded
 * separately in the order written, each product summed with one fused multiply-add per
 * term in ascending column order (the reading also used for the SBM field); the loss and
 * the gradient inner products accumulated in FP64.  Per step:
 *   f = J x;  h = f + b;  g = lambda_t x + h;  m' = alpha m - eta g;  y = x + m';
 *   x' = clip(y).   Reverse: ybar = xbar [|y| <= 1];  mu = ybar + alpha mu;
 *   xbar = ybar - eta (lambda_t mu + J mu).
 * Being piecewise smooth, the loss and its gradient can differ from the FP64 pass by
 * more than rounding where some |y| falls within rounding of 1 (a clip decided the other
 * way); the FP64 pass is the reference of the mathematics, this one of the arithmetic. */
static void matvec32(int fmt, int64_t n, const float *J, const int64_t *rp,
                     const int32_t *col, const float *w, const float *v, float *out)
{
    for (int64_t i = 0; i < n; ++i) {
        float acc = 0.0f;
        if (fmt == 0) {
            for (int64_t j = 0; j < n; ++j) acc = fmaf(J[i * n + j], v[j], acc);
        } else {
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k) acc = fmaf(w[k], v[col[k]], acc);
        }
        out[i] = acc;
    }
}

static double relaxed_grad32(int fmt, int64_t n, const float *J, const int64_t *rp,
                             const int32_t *col, const float *w, const float *b, int64_t nrep,
                             const float *x0, int64_t T, const float *lam, float eta,
                             float alpha, double norm, double *d_eta, double *d_alpha,
                             double *d_lam, float *xT)
{
    float *X = (float *)malloc(sizeof(float) * (size_t)((T + 1) * n));
    float *M = (float *)malloc(sizeof(float) * (size_t)((T + 1) * n));
    float *F = (float *)malloc(sizeof(float) * (size_t)((T + 1) * n));
    float *xbar = (float *)malloc(sizeof(float) * (size_t)n);
    float *mu = (float *)malloc(sizeof(float) * (size_t)n);
    float *ybar = (float *)malloc(sizeof(float) * (size_t)n);
    float *jmu = (float *)malloc(sizeof(float) * (size_t)n);
    double loss = 0.0;
    if (d_eta) *d_eta = 0.0;
    if (d_alpha) *d_alpha = 0.0;
    if (d_lam) for (int64_t t = 0; t < T; ++t) d_lam[t] = 0.0;

    for (int64_t r = 0; r < nrep; ++r) {
        memcpy(X, x0 + r * n, sizeof(float) * (size_t)n);
        memset(M, 0, sizeof(float) * (size_t)n);
        for (int64_t t = 0; t < T; ++t) {
            const float *x = X + t * n, *mm = M + t * n;
            float *f = F + t * n, *xn = X + (t + 1) * n, *mn = M + (t + 1) * n;
            matvec32(fmt, n, J, rp, col, w, x, f);
            for (int64_t i = 0; i < n; ++i) {
                const float h = f[i] + b[i];
                const float g = lam[t] * x[i] + h;
                const float mv = alpha * mm[i] - eta * g;
                const float y = x[i] + mv;
                mn[i] = mv;
                xn[i] = y > 1.0f ? 1.0f : (y < -1.0f ? -1.0f : y);
            }
        }
        const float *xt = X + T * n;
        float *ft = F + T * n;
        if (xT) memcpy(xT + r * n, xt, sizeof(float) * (size_t)n);
        matvec32(fmt, n, J, rp, col, w, xt, ft);
        double e = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            const double xv = xt[i], fv = ft[i], bv = b[i];
            e += 0.5 * xv * fv + bv * xv;
            xbar[i] = (float)(norm * (fv + bv));
            mu[i] = 0.0f;
        }
        loss += e * norm;
        if (!(d_eta || d_alpha || d_lam)) continue;
        for (int64_t t = T - 1; t >= 0; --t) {
            const float *x = X + t * n, *mm = M + t * n, *f = F + t * n;
            double se = 0.0, sa = 0.0, sl = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                const float h = f[i] + b[i];
                const float g = lam[t] * x[i] + h;
                const float mv = alpha * mm[i] - eta * g;
                const float y = x[i] + mv;
                ybar[i] = fabsf(y) <= 1.0f ? xbar[i] : 0.0f;
                mu[i] = ybar[i] + alpha * mu[i];
                se += (double)mu[i] * (double)(-g);
                sa += (double)mu[i] * (double)mm[i];
                sl += (double)mu[i] * (-(double)eta * (double)x[i]);
            }
            if (d_eta) *d_eta += se;
            if (d_alpha) *d_alpha += sa;
            if (d_lam) d_lam[t] += sl;
            matvec32(fmt, n, J, rp, col, w, mu, jmu);
            for (int64_t i = 0; i < n; ++i)
                xbar[i] = ybar[i] - eta * (lam[t] * mu[i] + jmu[i]);
        }
    }
    free(X); free(M); free(F); free(xbar); free(mu); free(ybar); free(jmu);
    return loss;
}

double orc_relaxed_grad_dense_f32(int64_t n, const float *J, const float *b, int64_t nrep,
                                  const float *x0, int64_t T, const float *lam, float eta,
                                  float alpha, double norm, double *d_eta, double *d_alpha,
                                  double *d_lam, float *xT)
{
    return relaxed_grad32(0, n, J, NULL, NULL, NULL, b, nrep, x0, T, lam, eta, alpha, norm,
                          d_eta, d_alpha, d_lam, xT);
}

double orc_relaxed_grad_csr_f32(int64_t n, const int64_t *rp, const int32_t *col,
                                const float *w, const float *b, int64_t nrep, const float *x0,
                                int64_t T, const float *lam, float eta, float alpha,
                                double norm, double *d_eta, double *d_alpha, double *d_lam,
                                float *xT)
{
    return relaxed_grad32(1, n, NULL, rp, col, w, b, nrep, x0, T, lam, eta, alpha, norm, d_eta,
                          d_alpha, d_lam, xT);
}

/* ---------------------------------------------------------------------------------------
 * Simulated Bifurcation Machine (App. B, SBM): Hamilton's equations of the oscillator
 * network, dq/dt = a0 p, dp/dt = -(q^2 + a0 - a(t)) q + c0 (J' q + h'), integrated by
 * symplectic Euler with step dt: every p is advanced from the positions of the step,
 * then every q from its new p.  The problem is given in the PA convention (minimise
 * H = 1/2 s^T J s + b^T s); SBM maximises 1/2 q^T J' q + h'^T q, so it runs on
 * (J', h') = (-J, -b), i.e. its force is -c0 (J q + b).  a(t) = a0 * t / T rises
 * linearly.  Every operation is one FP32 rounding, in this order:
 *   g = (sum_j J_ij q_j, one fused multiply-add per term, in ascending j) + b_i
 *   w = ((q q + a0) - a) q;   F = -w - c0 g;   p = p + dt F;   q = q + (dt a0) p
 * (dt a0 rounded once).  g_out, when given, receives g of the last step.
 * ------------------------------------------------------------------------------------- */
static void sbm_update_row(int64_t n, const float *g, float a, float a0, float c0, float dt,
                           float *q, float *p)
{
    const float adt = dt * a0;
    for (int64_t i = 0; i < n; ++i) {
        float qq = q[i] * q[i];
        float w = ((qq + a0) - a) * q[i];
        float cg = c0 * g[i];
        float force = -w - cg;
        float pn = p[i] + dt * force;
        p[i] = pn;
        q[i] = q[i] + adt * pn;
    }
}

void orc_sbm_steps_dense_f32(int64_t n, const float *J, const float *b, int64_t nrep,
                             float *q, float *p, int64_t t0, int64_t t1, int64_t T, float a0,
                             float c0, float dt, float *g_out)
{
    float *g = (float *)malloc(sizeof(float) * (size_t)n);
    for (int64_t r = 0; r < nrep; ++r) {
        float *qr = q + r * n, *pr = p + r * n;
        for (int64_t t = t0; t < t1; ++t) {
            const float a = a0 * ((float)t / (float)T);
            for (int64_t i = 0; i < n; ++i) {
                float acc = 0.0f;
                for (int64_t j = 0; j < n; ++j) acc = fmaf(J[i * n + j], qr[j], acc);
                g[i] = acc + b[i];
            }
            sbm_update_row(n, g, a, a0, c0, dt, qr, pr);
        }
        if (g_out && t1 > t0) memcpy(g_out + r * n, g, sizeof(float) * (size_t)n);
    }
    free(g);
}

/* CSR couplings (weights converted to float, entries in row order, no diagonal). */
void orc_sbm_steps_csr_f32(int64_t n, const int64_t *rp, const int32_t *col, const float *w,
                           const float *b, int64_t nrep, float *q, float *p, int64_t t0,
                           int64_t t1, int64_t T, float a0, float c0, float dt, float *g_out)
{
    float *g = (float *)malloc(sizeof(float) * (size_t)n);
    for (int64_t r = 0; r < nrep; ++r) {
        float *qr = q + r * n, *pr = p + r * n;
        for (int64_t t = t0; t < t1; ++t) {
            const float a = a0 * ((float)t / (float)T);
            for (int64_t i = 0; i < n; ++i) {
                float acc = 0.0f;
                for (int64_t k = rp[i]; k < rp[i + 1]; ++k) acc = fmaf(w[k], qr[col[k]], acc);
                g[i] = acc + b[i];
            }
            sbm_update_row(n, g, a, a0, c0, dt, qr, pr);
        }
        if (g_out && t1 > t0) memcpy(g_out + r * n, g, sizeof(float) * (size_t)n);
    }
    free(g);
}
