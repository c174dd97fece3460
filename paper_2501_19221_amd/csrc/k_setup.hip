// Set-up and scoring kernels: canonicalisation (App. A), validation, initial state,
// state layout copies, exact energies (eq. (1) / eq. (2)) and best-of-replica.
#include "qpa_internal.h"

#include <algorithm>
#include <type_traits>

#include <math.h>

namespace qpa {
namespace {

constexpr int WAVE = 64;

template <typename T> __device__ __forceinline__ T ld(const void *p, int64_t k) {
    return static_cast<const T *>(p)[k];
}

// Read element k of an array of caller dtype `dt` as double (exact for every dtype here).
__device__ __forceinline__ double load_as_double(const void *p, int32_t dt, int64_t k) {
    switch (dt) {
        case QPA_I8: return (double)ld<int8_t>(p, k);
        case QPA_I16: return (double)ld<int16_t>(p, k);
        case QPA_I32: return (double)ld<int32_t>(p, k);
        default: return (double)ld<float>(p, k);
    }
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Round-to-nearest-even of a finite float to bf16 (upper 16 bits).
__device__ __forceinline__ uint16_t bf16_rne(float v) {
    uint32_t u = __float_as_uint(v);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// ------------------------------------------------------------------ dense canonicalisation
// One wave per row i.  Integer values are carried in double, exact below 2^53.
template <typename TQ>
__global__ void __launch_bounds__(256) k_dense_rows(int64_t n, const TQ *__restrict__ Q,
                                                    const void *lin, int32_t lin_dt,
                                                    int32_t is_qubo, float *__restrict__ J_f32,
                                                    float *__restrict__ b_f32,
                                                    int64_t *__restrict__ b_i64,
                                                    double *__restrict__ b_f64,
                                                    double *__restrict__ row_abs,
                                                    double *__restrict__ row_max,
                                                    double *__restrict__ row_k,
                                                    CanonScalars *sc) {
    const int lane = threadIdx.x % WAVE;
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    if (i >= n) return;
    const TQ *row = Q + i * n;
    double sum = 0.0, sabs = 0.0, smax = 0.0, diag = 0.0;
    for (int64_t j = lane; j < n; j += WAVE) {
        double q = (double)row[j];
        sum += q;
        if (j == i) {
            diag = q;
        } else {
            sabs += fabs(q);
            smax = fmax(smax, fabs(q));
        }
        if (J_f32) J_f32[i * n + j] = (j == i) ? 0.0f : (float)row[j];
    }
    sum = wave_sum(sum);
    sabs = wave_sum(sabs);
    smax = wave_max(smax);
    diag = wave_sum(diag);
    if (lane == 0) {
        double c = lin ? load_as_double(lin, lin_dt, i) : 0.0;
        if (!is_qubo && diag != 0.0) atomicOr(&sc->flags, (int32_t)FLAG_ASYM);
        double bx = (is_qubo ? sum : 0.0) + c;
        b_f32[i] = (float)bx;
        if (b_i64) b_i64[i] = (int64_t)bx;
        b_f64[i] = bx;
        row_abs[i] = sabs + fabs(bx);
        row_max[i] = smax;
        // contribution to 2K = 1^T Q 1 + tr Q + 2 1^T c  (QUBO only)
        row_k[i] = is_qubo ? (sum + diag + 2.0 * c) : 0.0;
    }
}

// Symmetry: compare the 32x32 tiles (by, bx) and (bx, by) through LDS.
template <typename TQ>
__global__ void __launch_bounds__(256) k_dense_sym(int64_t n, const TQ *__restrict__ Q,
                                                   CanonScalars *sc) {
    __shared__ TQ tile[32][33];
    const int64_t bx = blockIdx.x, by = blockIdx.y;
    if (bx > by) return;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;   // 32 x 8
    // load tile (bx, by) transposed: element (r = by*32 + ..., c = bx*32 + ...)
    for (int k = ty; k < 32; k += 8) {
        int64_t r = bx * 32 + k, c = by * 32 + tx;
        tile[tx][k] = (r < n && c < n) ? Q[r * n + c] : TQ(0);
    }
    __syncthreads();
    int bad = 0;
    for (int k = ty; k < 32; k += 8) {
        int64_t r = by * 32 + k, c = bx * 32 + tx;
        if (r < n && c < n) bad |= (Q[r * n + c] != tile[k][tx]);
    }
    if (bad) atomicOr(&sc->flags, (int32_t)FLAG_ASYM);
}

// Large instances reduce the per-row partials in two launches: k_canon_part gives each of
// P workgroups a contiguous range of rows and writes (max |row|, max |J|, sum K as double,
// sum K as int64) to parts[4 p ..]; k_canon_finalize then reduces those P values (both in
// a fixed order, so the scalars are reproducible); P = ceil(n / CANON_ROWS_PER_PART),
// at most CANON_PARTS.

__global__ void __launch_bounds__(1024) k_canon_part(int64_t n, int64_t rows,
                                                     const double *row_abs,
                                                     const double *row_max,
                                                     const double *row_k, double *parts) {
    __shared__ double s_abs[1024 / WAVE], s_max[1024 / WAVE], s_k[1024 / WAVE];
    __shared__ int64_t s_ki[1024 / WAVE];
    const int64_t i0 = (int64_t)blockIdx.x * rows;
    const int64_t i1 = i0 + rows < n ? i0 + rows : n;
    double a = 0.0, mx = 0.0, kf = 0.0;
    int64_t ki = 0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        a = fmax(a, row_abs[i]);
        if (row_max) mx = fmax(mx, row_max[i]);
        kf += row_k[i];
        ki += (int64_t)row_k[i];
    }
    a = wave_max(a);
    mx = wave_max(mx);
    kf = wave_sum(kf);
    ki = wave_sum_i64(ki);
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    if (lane == 0) {
        s_abs[w] = a;
        s_max[w] = mx;
        s_k[w] = kf;
        s_ki[w] = ki;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double A = 0.0, M = 0.0, Kf = 0.0;
        int64_t Ki = 0;
        for (int k = 0; k < (int)(blockDim.x / WAVE); ++k) {
            A = fmax(A, s_abs[k]);
            M = fmax(M, s_max[k]);
            Kf += s_k[k];
            Ki += s_ki[k];
        }
        double *pp = parts + 4 * blockIdx.x;
        pp[0] = A;
        pp[1] = M;
        pp[2] = Kf;
        pp[3] = __longlong_as_double(Ki);
    }
}

// Single block: reduce the per-row partials (or, with `parts`, the P partials of
// k_canon_part) into the scalars.
__device__ __forceinline__ void canon_finalize_body(int64_t n, const double *row_abs,
                                                    const double *row_max, const double *row_k,
                                                    const double *parts, int32_t is_int,
                                                    CanonScalars *sc, CanonScalars *mirror) {
    __shared__ double s_abs[1024 / WAVE], s_max[1024 / WAVE], s_k[1024 / WAVE];
    __shared__ int64_t s_ki[1024 / WAVE];
    double a = 0.0, mx = 0.0, kf = 0.0;
    int64_t ki = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        if (parts) {
            a = fmax(a, parts[4 * i]);
            mx = fmax(mx, parts[4 * i + 1]);
            kf += parts[4 * i + 2];
            ki += __double_as_longlong(parts[4 * i + 3]);
        } else {
            a = fmax(a, row_abs[i]);
            if (row_max) mx = fmax(mx, row_max[i]);
            kf += row_k[i];
            ki += (int64_t)row_k[i];
        }
    }
    a = wave_max(a);
    mx = wave_max(mx);
    kf = wave_sum(kf);
    ki = wave_sum_i64(ki);
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    if (lane == 0) {
        s_abs[w] = a;
        s_max[w] = mx;
        s_k[w] = kf;
        s_ki[w] = ki;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double A = 0.0, M = 0.0, Kf = 0.0;
        int64_t Ki = 0;
        for (int k = 0; k < (int)(blockDim.x / WAVE); ++k) {
            A = fmax(A, s_abs[k]);
            M = fmax(M, s_max[k]);
            Kf += s_k[k];
            Ki += s_ki[k];
        }
        sc->max_row = A;
        sc->max_abs = M;
        sc->K_f64 = 0.5 * Kf;
        sc->K_i64 = Ki / 2;
        // the flags of the earlier kernels, read atomically, plus the range bit
        const int32_t add = (is_int && A >= 16777216.0) ? (int32_t)FLAG_RANGE : 0;
        const int32_t flags = atomicOr(&sc->flags, add) | add;
        int e = 0;
        if (M > 0.0) {
            e = (int)ceil(log2(M));
            // guard the rounding of log2 near powers of two
            while (ldexp(1.0, e) < M) ++e;
            while (e > -126 && ldexp(1.0, e - 1) >= M) --e;
        }
        sc->exp2 = e;
        sc->scale = ldexpf(1.0f, e);
        sc->inv_scale = ldexpf(1.0f, -e);
        if (mirror) {            // a copy in a contiguous array of a batch's instances
            CanonScalars c;
            c.K_i64 = Ki / 2;
            c.K_f64 = 0.5 * Kf;
            c.scale = ldexpf(1.0f, e);
            c.inv_scale = ldexpf(1.0f, -e);
            c.flags = flags;
            c.exp2 = e;
            c.max_row = A;
            c.max_abs = M;
            *mirror = c;
        }
    }
}

__global__ void __launch_bounds__(1024) k_canon_finalize(int64_t n, const double *row_abs,
                                                         const double *row_max,
                                                         const double *row_k,
                                                         const double *parts, int32_t is_int,
                                                         CanonScalars *sc, CanonScalars *mirror) {
    canon_finalize_body(n, row_abs, row_max, row_k, parts, is_int, sc, mirror);
}

__global__ void __launch_bounds__(1024) k_canon_finalize_batch(const CanonTask *__restrict__ tasks) {
    const CanonTask &t = tasks[blockIdx.y];
    canon_finalize_body(t.n, t.row_abs, t.row_max, t.row_k, nullptr, t.is_int, t.sc, t.mirror);
}

template <typename TQ>
__global__ void __launch_bounds__(256) k_dense_bf16(int64_t n, int64_t npad,
                                                    const TQ *__restrict__ Q,
                                                    const CanonScalars *sc,
                                                    uint16_t *__restrict__ Jb) {
    const float inv = sc->inv_scale;
    const int64_t total = npad * npad;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = k / npad, j = k - i * npad;
        uint16_t v = 0;
        if (i < n && j < n && i != j) v = bf16_rne((float)Q[i * n + j] * inv);
        Jb[k] = v;
    }
}

// ------------------------------------------------------------------ CSR canonicalisation
template <typename TW, typename TI>
__global__ void __launch_bounds__(256) k_csr_rows(int64_t n, int64_t nnz,
                                                  const int32_t *__restrict__ rp,
                                                  const TI *__restrict__ col,
                                                  const TW *__restrict__ w, const void *lin,
                                                  int32_t lin_dt, int32_t is_qubo,
                                                  float *__restrict__ b_f32,
                                                  int64_t *__restrict__ b_i64,
                                                  double *__restrict__ b_f64,
                                                  double *__restrict__ row_abs,
                                                  double *__restrict__ row_max,
                                                  double *__restrict__ row_k,
                                                  CanonScalars *sc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t flags = 0;
    double smax = 0.0;
    const int64_t k0 = rp[i], k1 = rp[i + 1];
    if (i == 0 && k0 != 0) flags |= FLAG_SHAPE;
    if (i == n - 1 && k1 != nnz) flags |= FLAG_SHAPE;
    double sum = 0.0, sabs = 0.0, diag = 0.0;
    if (k0 > k1 || k0 < 0 || k1 > nnz) {
        flags |= FLAG_SHAPE;
    } else {
        int64_t prev = -1;
        for (int64_t k = k0; k < k1; ++k) {
            int64_t j = (int64_t)col[k];
            double v = (double)w[k];
            if (j < 0 || j >= n) {
                flags |= FLAG_SHAPE;
                continue;
            }
            if (j <= prev) flags |= FLAG_UNSORTED;
            prev = j;
            sum += v;
            if (j == i) {
                diag += v;
                if (!is_qubo) flags |= FLAG_ASYM;
                continue;
            }
            sabs += fabs(v);
            smax = fmax(smax, fabs(v));
            // symmetric partner (j, i) with the same weight: binary search in row j
            int64_t lo = rp[j], hi = rp[j + 1] - 1;
            bool found = false;
            while (lo <= hi && lo >= 0 && hi < nnz) {
                int64_t mid = (lo + hi) >> 1;
                int64_t cm = (int64_t)col[mid];
                if (cm == i) {
                    found = ((double)w[mid] == v);
                    break;
                }
                if (cm < i) lo = mid + 1;
                else hi = mid - 1;
            }
            if (!found) flags |= FLAG_ASYM;
        }
    }
    double c = lin ? load_as_double(lin, lin_dt, i) : 0.0;
    double bx = (is_qubo ? sum : 0.0) + c;
    b_f32[i] = (float)bx;
    if (b_i64) b_i64[i] = (int64_t)bx;
    b_f64[i] = bx;
    row_abs[i] = sabs + fabs(bx);
    if (row_max) row_max[i] = smax;
    row_k[i] = is_qubo ? (sum + diag + 2.0 * c) : 0.0;
    if (flags) atomicOr(&sc->flags, flags);
}

// Integer CSR rows with many entries: one wave per row, the row's entries split over the
// lanes (the symmetric-partner searches run in parallel).  Outputs as k_csr_rows; every
// sum is an exact integer, so the order of the reduction does not matter.
template <typename TW, typename TI>
__device__ __forceinline__ void csr_rows_wave_body(int64_t i, int64_t n, int64_t nnz,
                                                   const int32_t *__restrict__ rp,
                                                   const TI *__restrict__ col,
                                                   const TW *__restrict__ w, const void *lin,
                                                   int32_t lin_dt, int32_t is_qubo,
                                                   float *__restrict__ b_f32,
                                                   int64_t *__restrict__ b_i64,
                                                   double *__restrict__ b_f64,
                                                   double *__restrict__ row_abs,
                                                   double *__restrict__ row_max,
                                                   double *__restrict__ row_k,
                                                   CanonScalars *sc) {
    const int lane = threadIdx.x % WAVE;
    if (i >= n) return;                        // uniform per wave
    int32_t flags = 0;
    const int64_t k0 = rp[i], k1 = rp[i + 1];
    if (i == 0 && k0 != 0) flags |= FLAG_SHAPE;
    if (i == n - 1 && k1 != nnz) flags |= FLAG_SHAPE;
    int64_t sum = 0, sabs = 0, diag = 0, smax = 0;
    if (k0 > k1 || k0 < 0 || k1 > nnz) {
        flags |= FLAG_SHAPE;
    } else {
        for (int64_t k = k0 + lane; k < k1; k += WAVE) {
            const int64_t j = (int64_t)col[k];
            const int64_t v = (int64_t)w[k];
            if (j < 0 || j >= n) {
                flags |= FLAG_SHAPE;
                continue;
            }
            if (k > k0 && (int64_t)col[k - 1] >= j) flags |= FLAG_UNSORTED;
            sum += v;
            if (j == i) {
                diag += v;
                if (!is_qubo) flags |= FLAG_ASYM;
                continue;
            }
            const int64_t av = v < 0 ? -v : v;
            sabs += av;
            smax = av > smax ? av : smax;
            int64_t lo = rp[j], hi = rp[j + 1] - 1;
            bool found = false;
            while (lo <= hi && lo >= 0 && hi < nnz) {
                const int64_t mid = (lo + hi) >> 1;
                const int64_t cm = (int64_t)col[mid];
                if (cm == i) {
                    found = ((int64_t)w[mid] == v);
                    break;
                }
                if (cm < i) lo = mid + 1;
                else hi = mid - 1;
            }
            if (!found) flags |= FLAG_ASYM;
        }
    }
    sum = wave_sum_i64(sum);
    sabs = wave_sum_i64(sabs);
    diag = wave_sum_i64(diag);
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        const int64_t other = __shfl_xor(smax, o);
        smax = other > smax ? other : smax;
        flags |= __shfl_xor(flags, o);
    }
    if (lane != 0) return;
    const double c = lin ? load_as_double(lin, lin_dt, i) : 0.0;
    const double bx = (is_qubo ? (double)sum : 0.0) + c;
    b_f32[i] = (float)bx;
    if (b_i64) b_i64[i] = (int64_t)bx;
    b_f64[i] = bx;
    row_abs[i] = (double)sabs + fabs(bx);
    if (row_max) row_max[i] = (double)smax;
    row_k[i] = is_qubo ? ((double)sum + (double)diag + 2.0 * c) : 0.0;
    if (flags) atomicOr(&sc->flags, flags);
}

template <typename TW, typename TI>
__global__ void __launch_bounds__(256) k_csr_rows_wave(int64_t n, int64_t nnz,
                                                       const int32_t *__restrict__ rp,
                                                       const TI *__restrict__ col,
                                                       const TW *__restrict__ w, const void *lin,
                                                       int32_t lin_dt, int32_t is_qubo,
                                                       float *__restrict__ b_f32,
                                                       int64_t *__restrict__ b_i64,
                                                       double *__restrict__ b_f64,
                                                       double *__restrict__ row_abs,
                                                       double *__restrict__ row_max,
                                                       double *__restrict__ row_k,
                                                       CanonScalars *sc) {
    csr_rows_wave_body<TW, TI>((int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE, n, nnz,
                               rp, col, w, lin, lin_dt, is_qubo, b_f32, b_i64, b_f64, row_abs,
                               row_max, row_k, sc);
}

// Batched canonicalisation (instance blockIdx.y of the table): clear the scalars, the
// row pass, the finalisation; each as the single-instance kernels do it.
__global__ void __launch_bounds__(64) k_canon_zero_batch(const CanonTask *__restrict__ tasks) {
    if (threadIdx.x == 0) *tasks[blockIdx.y].sc = CanonScalars{};
}

template <typename TW, typename TI>
__global__ void __launch_bounds__(256) k_csr_rows_wave_batch(const CanonTask *__restrict__ tasks) {
    const CanonTask &t = tasks[blockIdx.y];
    csr_rows_wave_body<TW, TI>((int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE, t.n,
                               t.nnz, t.rp, static_cast<const TI *>(t.col),
                               static_cast<const TW *>(t.w), t.lin, t.lin_dt, t.is_qubo,
                               t.b_f32, t.b_i64, t.b_f64, t.row_abs, t.row_max, t.row_k, t.sc);
}

// ------------------------------------------------------------------ initial state
// Replica r, variable i: u = top 24 bits of SplitMix64 output number r*n + i + 1.
__device__ __forceinline__ uint64_t splitmix_output(uint64_t seed, uint64_t k) {
    uint64_t z = seed + k * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// x0 of replica r, variable i (0 in the padding past R or n).
__device__ __forceinline__ float init_x(uint64_t seed, float sigma0, int64_t n, int64_t R,
                                        int64_t r, int64_t i) {
    float xv = 0.0f;
    if (r < R && i < n) {
        uint64_t top = splitmix_output(seed, (uint64_t)(r * n + i) + 1u) >> 40;
        float u = __fmul_rn((float)top, 1.0f / 16777216.0f);
        float v = __fsub_rn(__fmul_rn(2.0f, u), 1.0f);
        xv = __fmul_rn(sigma0, v);
    }
    return xv;
}

__global__ void __launch_bounds__(256) k_init_state(int64_t n, int64_t R, uint64_t seed,
                                                    float sigma0, float *__restrict__ x,
                                                    float *__restrict__ m, int64_t ld_r,
                                                    int64_t ld_i, int64_t Rpad, int64_t npad) {
    const int64_t total = Rpad * npad;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        int64_t r, i;
        if (ld_i == 1) {          // replica-major: consecutive threads walk variables
            r = k / npad;
            i = k - r * npad;
        } else {                  // variable-major: consecutive threads walk replicas
            i = k / Rpad;
            r = k - i * Rpad;
        }
        const float xv = init_x(seed, sigma0, n, R, r, i);
        x[r * ld_r + i * ld_i] = xv;
        m[r * ld_r + i * ld_i] = 0.0f;
    }
}

// Batched set-up of int8 dense slots (instance blockIdx.y of the table): x0 and m0 as
// k_init_state in the [Rp][np] layout, the byte spins of x0 as the int8 tile kernel
// reads them (chunk-major: element (r, i) at (i / C) * Rp * C + r * C + i % C, C =
// MF_NPAD, 0xFF for a negative x), and the field padded to np.
__global__ void __launch_bounds__(256) k_slot_init_batch(const SlotInitTask *__restrict__ tasks,
                                                         float sigma0) {
    const SlotInitTask &t = tasks[blockIdx.y];
    const int64_t total = t.Rp * t.np;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = k / t.np, i = k - r * t.np;
        const float xv = init_x(t.seed, sigma0, t.n, t.R, r, i);
        t.x[k] = xv;
        t.m[k] = 0.0f;
        t.s8[(i / MF_NPAD) * t.Rp * MF_NPAD + r * MF_NPAD + i % MF_NPAD] =
            xv < 0.0f ? (uint8_t)0xFF : (uint8_t)0x01;
        if (r == 0) t.bfp[i] = i < t.n ? t.bf[i] : 0.0f;
    }
}

__global__ void __launch_bounds__(256) k_copy_state(int64_t n, int64_t R, const float *src,
                                                    int64_t s_ld_r, int64_t s_ld_i,
                                                    float *dst, int64_t d_ld_r,
                                                    int64_t d_ld_i) {
    const int64_t total = R * n;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        int64_t r, i;
        if (d_ld_i == 1) {
            r = k / n;
            i = k - r * n;
        } else {
            i = k / R;
            r = k - i * R;
        }
        dst[r * d_ld_r + i * d_ld_i] = src[r * s_ld_r + i * s_ld_i];
    }
}

__device__ __forceinline__ void export_spins_body(int64_t n, int64_t R, const float *x,
                                                  int64_t ld_r, int64_t ld_i, int8_t *spins) {
    const int64_t total = R * n;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = k / n, i = k - r * n;
        spins[k] = (x[r * ld_r + i * ld_i] >= 0.0f) ? (int8_t)1 : (int8_t)-1;
    }
}

__global__ void __launch_bounds__(256) k_pad_f32(int64_t n, int64_t np, const float *src,
                                                 float *dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = i < n ? src[i] : 0.0f;
}

__global__ void __launch_bounds__(256) k_export_spins(int64_t n, int64_t R, const float *x,
                                                      int64_t ld_r, int64_t ld_i,
                                                      int8_t *spins) {
    export_spins_body(n, R, x, ld_r, ld_i, spins);
}

// Batched scoring: instance blockIdx.y of the task table, the same work per instance as
// the single-instance kernels (one launch per kind instead of one per instance).
__global__ void __launch_bounds__(256) k_export_spins_batch(const ScoreTask *__restrict__ tasks) {
    const ScoreTask &t = tasks[blockIdx.y];
    export_spins_body(t.n, t.R, t.x, t.ld_r, 1, t.spins);
}

// ------------------------------------------------------------------ energies
// H(s) = sum_{i<j} J_ij s_i s_j + sum_i b_i s_i (eq. (2)); for a QUBO the objective is
// E = (H + K) / 2 with the canonical (J, b, K).
constexpr int ER = 16;

// Dense: thread = replica.  A workgroup owns EROWS rows i and walks the columns in
// chunks of 8.  For each row and chunk it builds the table of all 256 signed sums
//   T_i[B] = sum_{k<8} J_{i,8c+k} (bit k of B ? -1 : +1)     (diagonal excluded)
// (from two 16-entry half tables), after which replica r's row sum over the chunk is one
// lookup T_i[B_r] with B_r its 8 sign bits there.  Per replica it accumulates
//   sum_i s_i (J s)_i + 2 sum_i s_i b_i = 2 H(s)
// over its rows; the tables are FP64 (exact for integer couplings, whose rows are
// validated below 2^24).  Spins arrive bit-packed per replica (k_spin_rowbits).
constexpr int EROWS = 16;

__global__ void __launch_bounds__(256) k_spin_rowbits(int64_t n, int64_t R, int64_t nw,
                                                      const int8_t *__restrict__ s,
                                                      uint64_t *__restrict__ bits) {
    // one wave per replica; bit i%64 of word i/64 set <=> spin i is -1
    const int lane = threadIdx.x & 63;
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (r >= R) return;
    for (int64_t w = 0; w < nw; ++w) {
        const int64_t i = 64 * w + lane;
        const uint64_t word = __ballot(i < n && s[r * n + i] < 0);
        if (lane == 0) bits[r * nw + w] = word;
    }
}

template <typename TQ>
__global__ void __launch_bounds__(1024) k_energy_dense(int64_t n, int64_t nw,
                                                       const TQ *__restrict__ Q,
                                                       const int64_t *__restrict__ b_i64,
                                                       const double *__restrict__ b_f64,
                                                       const uint64_t *__restrict__ bits,
                                                       int64_t R, double *__restrict__ partial) {
    __shared__ double T[EROWS][256];
    __shared__ double N[EROWS][2][16];
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * EROWS;
    for (int64_t r0 = 0; r0 < R; r0 += 1024) {
        const int64_t r = r0 + t;
        const bool live = r < R;
        const uint64_t *br = bits + (live ? r : 0) * nw;
        double h[EROWS];
#pragma unroll
        for (int k = 0; k < EROWS; ++k) h[k] = 0.0;
        uint64_t word = 0;
        for (int64_t c = 0; c < n; c += 8) {
            if (t < EROWS * 32) {                 // half tables: 4 columns each
                const int row = t >> 5, half = (t >> 4) & 1, e = t & 15;
                const int64_t i = i0 + row;
                double v = 0.0;
                if (i < n) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int64_t j = c + 4 * half + k;
                        const double q = (j < n && j != i) ? (double)Q[i * n + j] : 0.0;
                        v += ((e >> k) & 1) ? -q : q;
                    }
                }
                N[row][half][e] = v;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < EROWS / 4; ++u) {
                const int idx = t + 1024 * u, row = idx >> 8, e = idx & 255;
                T[row][e] = N[row][0][e & 15] + N[row][1][e >> 4];
            }
            __syncthreads();
            if ((c & 63) == 0 && live) word = br[c >> 6];
            const int B = (int)((word >> (c & 63)) & 0xFFu);
#pragma unroll
            for (int k = 0; k < EROWS; ++k) h[k] += T[k][B];
        }
        if (live) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < EROWS; ++k) {
                const int64_t i = i0 + k;
                if (i < n) {
                    const bool neg = (br[i >> 6] >> (i & 63)) & 1u;
                    const double bi = b_i64 ? (double)b_i64[i] : b_f64[i];
                    const double term = h[k] + 2.0 * bi;
                    acc += neg ? -term : term;
                }
            }
            partial[(int64_t)blockIdx.x * R + r] = acc;
        }
        __syncthreads();
    }
}

// CSR: one thread per row, replicas r0 .. r0+ER.
template <typename TW, typename TI, bool INT>
__global__ void __launch_bounds__(256) k_energy_csr(int64_t n, const int32_t *__restrict__ rp,
                                                    const TI *__restrict__ col,
                                                    const TW *__restrict__ w,
                                                    const int64_t *__restrict__ b_i64,
                                                    const double *__restrict__ b_f64,
                                                    const int8_t *__restrict__ s, int64_t R,
                                                    double *__restrict__ partial) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.y * ER;
    __shared__ double red[256 / WAVE][ER];
    double contrib[ER];
#pragma unroll
    for (int q = 0; q < ER; ++q) contrib[q] = 0.0;
    if (i < n) {
        const int64_t k0 = rp[i], k1 = rp[i + 1];
#pragma unroll
        for (int q = 0; q < ER; ++q) {
            int64_t r = r0 + q;
            if (r >= R) continue;
            const int8_t *sr = s + r * n;
            int64_t di = 0;
            double df = 0.0;
            for (int64_t k = k0; k < k1; ++k) {
                int64_t j = (int64_t)col[k];
                if (INT ? (j <= i) : (j == i)) continue;   // integer: each pair once
                if (INT) di += (sr[j] > 0) ? (int64_t)w[k] : -(int64_t)w[k];
                else df += (sr[j] > 0) ? (double)w[k] : -(double)w[k];
            }
            double si = (double)sr[i];
            if (INT) contrib[q] = si * ((double)di + (double)b_i64[i]);
            else contrib[q] = si * (0.5 * df + b_f64[i]);
        }
    }
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
#pragma unroll
    for (int q = 0; q < ER; ++q) {
        double v = wave_sum(contrib[q]);
        if (lane == 0) red[wv][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < ER) {
        int q = threadIdx.x;
        int64_t r = r0 + q;
        if (r < R) {
            double v = 0.0;
            for (int k = 0; k < (int)(blockDim.x / WAVE); ++k) v += red[k][q];
            partial[(int64_t)blockIdx.x * R + r] = v;
        }
    }
}

// CSR, integer couplings, rows with many entries: one wave per row, the row's entries
// split over the lanes; replicas r0 .. r0+ER.  Same partial sums as k_energy_csr (each
// pair once, exact integers), with 4 rows per block.
template <typename TW, typename TI>
__device__ __forceinline__ void energy_csr_wave_body(int64_t n, const int32_t *__restrict__ rp,
                                                     const TI *__restrict__ col,
                                                     const TW *__restrict__ w,
                                                     const int64_t *__restrict__ b_i64,
                                                     const int8_t *__restrict__ s, int64_t R,
                                                     double *__restrict__ partial, int64_t bx,
                                                     int64_t by) {
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    const int64_t i = bx * (256 / WAVE) + wv;
    const int64_t r0 = by * ER;
    __shared__ double red[256 / WAVE][ER];
    int64_t di[ER];
#pragma unroll
    for (int q = 0; q < ER; ++q) di[q] = 0;
    if (i < n) {
        const int64_t k1 = rp[i + 1];
        for (int64_t k = rp[i] + lane; k < k1; k += WAVE) {
            const int64_t j = (int64_t)col[k];
            if (j <= i) continue;                 // each pair once
            const int64_t wk = (int64_t)w[k];
#pragma unroll
            for (int q = 0; q < ER; ++q) {
                const int64_t r = r0 + q < R ? r0 + q : R - 1;
                di[q] += (s[r * n + j] > 0) ? wk : -wk;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < ER; ++q) {
        const int64_t d = wave_sum_i64(di[q]);
        if (lane == 0) {
            double v = 0.0;
            const int64_t r = r0 + q;
            if (i < n && r < R) v = (double)s[r * n + i] * ((double)d + (double)b_i64[i]);
            red[wv][q] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < ER) {
        const int q = threadIdx.x;
        const int64_t r = r0 + q;
        if (r < R) {
            double v = 0.0;
            for (int k = 0; k < 256 / WAVE; ++k) v += red[k][q];
            partial[bx * R + r] = v;
        }
    }
}

template <typename TW, typename TI>
__global__ void __launch_bounds__(256) k_energy_csr_wave(int64_t n,
                                                         const int32_t *__restrict__ rp,
                                                         const TI *__restrict__ col,
                                                         const TW *__restrict__ w,
                                                         const int64_t *__restrict__ b_i64,
                                                         const int8_t *__restrict__ s, int64_t R,
                                                         double *__restrict__ partial) {
    energy_csr_wave_body<TW, TI>(n, rp, col, w, b_i64, s, R, partial, blockIdx.x, blockIdx.y);
}

// Batched energies of integer CSR instances (n <= EBITS_MAX_N) from bit-packed spins:
// the same partial sums as the wave-per-row kernel (each pair once, exact integers),
// over blocks of EB_ROWS rows.  k_spin_words_batch writes each replica's sign bits once
// (bit i % 64 of word i / 64 set <=> not x_i >= 0, i.e. spin -1); an energy block stages the
// words of 64 replicas in LDS as words[i / 64][replica], a wave takes a row with lane =
// replica and walks the row's entries past the diagonal in pieces of 64 (loaded by the
// lanes, then broadcast one at a time), so that no spin is fetched from memory per entry.
__global__ void __launch_bounds__(256) k_spin_words_batch(const ScoreTask *__restrict__ tasks) {
    const ScoreTask &t = tasks[blockIdx.y];
    const int64_t nw = (t.n + 63) / 64, total = t.R * nw;
    const int lane = threadIdx.x & 63;
    const int64_t step = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; p < total;
         p += step) {
        const int64_t r = p / nw, i = 64 * (p - r * nw) + lane;
        // spin -1 exactly where the export writes -1: not (x >= 0)
        const uint64_t word = __ballot(i < t.n && !(t.x[r * t.ld_r + i] >= 0.0f));
        if (lane == 0) t.words[p] = word;
    }
}

template <typename TW, typename TI>
__global__ void __launch_bounds__(256) k_energy_bits_batch(const ScoreTask *__restrict__ tasks) {
    // rows padded by one word: the staging writes (consecutive threads on consecutive
    // rows) then fall in different banks
    __shared__ uint64_t words[EBITS_MAX_N / 64][64 + 1];
    __shared__ int64_t red[4][64];
    const ScoreTask &t = tasks[blockIdx.y];
    const int64_t n = t.n, R = t.R, nw = (n + 63) / 64;
    const int64_t i0 = (int64_t)blockIdx.x * EB_ROWS;
    if (i0 >= n) return;                          // uniform per block
    const TI *__restrict__ col = static_cast<const TI *>(t.col);
    const TW *__restrict__ w = static_cast<const TW *>(t.w);
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t r0 = 0; r0 < R; r0 += 64) {
        __syncthreads();                          // the previous group is no longer read
        for (int64_t q = threadIdx.x; q < 64 * nw; q += blockDim.x) {
            const int64_t rr = q / nw, wd = q - rr * nw;
            words[wd][rr] = r0 + rr < R ? t.words[(r0 + rr) * nw + wd] : 0ull;
        }
        __syncthreads();
        int64_t acc = 0;
        for (int e = wv; e < EB_ROWS; e += 4) {
            const int64_t i = i0 + e;
            if (i >= n) break;
            // first entry past the diagonal (the columns of a row are sorted)
            int64_t lo = t.rp[i], hi = t.rp[i + 1];
            const int64_t k1 = hi;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if ((int64_t)col[mid] <= i) lo = mid + 1;
                else hi = mid;
            }
            int32_t d = 0;
            for (int64_t kb = lo; kb < k1; kb += 64) {
                const int cnt = (int)(k1 - kb < 64 ? k1 - kb : 64);
                int32_t cj = 0, cw = 0;
                if (lane < cnt) {
                    cj = (int32_t)col[kb + lane];
                    cw = (int32_t)w[kb + lane];
                }
                for (int c = 0; c < cnt; ++c) {
                    const int32_t j = __builtin_amdgcn_readlane(cj, c);
                    const int32_t wj = __builtin_amdgcn_readlane(cw, c);
                    d += ((words[j >> 6][lane] >> (j & 63)) & 1ull) ? -wj : wj;
                }
            }
            const int64_t v = (int64_t)d + t.b_i64[i];
            acc += ((words[i >> 6][lane] >> (i & 63)) & 1ull) ? -v : v;
        }
        red[wv][lane] = acc;
        __syncthreads();
        if (threadIdx.x < 64 && r0 + (int64_t)threadIdx.x < R) {
            const int q = threadIdx.x;
            t.partial[(int64_t)blockIdx.x * R + r0 + q] =
                (double)(red[0][q] + red[1][q] + red[2][q] + red[3][q]);
        }
    }
}

// energy[r] = sum over blocks of partial[b][r] (fixed order), then the QUBO constant.
// For integer instances the partials are exact integers (< 2^53) and the total is taken
// in int64.
// One wave per replica: lane l sums partials l, l + 64, ... in order, then a fixed
// shuffle tree (deterministic; exact int64 sums for integer couplings).
// twice: the partials sum to 2 H (dense kernel) instead of H.
__device__ __forceinline__ void energy_finalize_body(int64_t R, int64_t nblk,
                                                     const double *__restrict__ partial,
                                                     int32_t is_int, int32_t is_qubo,
                                                     int32_t twice, const CanonScalars *sc,
                                                     int64_t *__restrict__ e_i64,
                                                     double *__restrict__ e_f64) {
    const int lane = threadIdx.x & 63;
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (r >= R) return;
    if (is_int) {
        int64_t H = 0;
        for (int64_t b = lane; b < nblk; b += 64) H += (int64_t)partial[b * R + r];
        for (int o = 32; o > 0; o >>= 1) H += __shfl_xor(H, o);
        if (lane) return;
        if (twice) H /= 2;
        int64_t E = is_qubo ? (H + sc->K_i64) / 2 : H;
        if (e_i64) e_i64[r] = E;
        e_f64[r] = (double)E;
    } else {
        double H = 0.0;
        for (int64_t b = lane; b < nblk; b += 64) H += partial[b * R + r];
        for (int o = 32; o > 0; o >>= 1) H += __shfl_xor(H, o);
        if (lane) return;
        if (twice) H *= 0.5;
        e_f64[r] = is_qubo ? 0.5 * (H + sc->K_f64) : H;
    }
}

__global__ void __launch_bounds__(256) k_energy_finalize(int64_t R, int64_t nblk,
                                                         const double *__restrict__ partial,
                                                         int32_t is_int, int32_t is_qubo,
                                                         int32_t twice, const CanonScalars *sc,
                                                         int64_t *__restrict__ e_i64,
                                                         double *__restrict__ e_f64) {
    energy_finalize_body(R, nblk, partial, is_int, is_qubo, twice, sc, e_i64, e_f64);
}

__global__ void __launch_bounds__(256) k_energy_finalize_batch(const ScoreTask *__restrict__ tasks) {
    const ScoreTask &t = tasks[blockIdx.y];
    energy_finalize_body(t.R, t.nblk, t.partial, 1, t.is_qubo, 0, t.sc, t.e_i64, t.e_f64);
}

__device__ __forceinline__ void argmin_body(int64_t R, const int64_t *e_i64,
                                            const double *e_f64, int32_t *best) {
    __shared__ double sv[1024];
    __shared__ int64_t si[1024];
    __shared__ int64_t sv_i[1024];
    double bv = INFINITY;
    int64_t bvi = INT64_MAX;
    int64_t bi = INT64_MAX;
    for (int64_t r = threadIdx.x; r < R; r += blockDim.x) {
        if (e_i64) {
            int64_t v = e_i64[r];
            if (v < bvi || (v == bvi && r < bi)) {
                bvi = v;
                bi = r;
            }
        } else {
            double v = e_f64[r];
            if (v < bv || (v == bv && r < bi) || bi == INT64_MAX) {
                bv = v;
                bi = r;
            }
        }
    }
    sv[threadIdx.x] = bv;
    sv_i[threadIdx.x] = bvi;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            int a = threadIdx.x, b = threadIdx.x + o;
            bool take;
            if (e_i64) take = sv_i[b] < sv_i[a] || (sv_i[b] == sv_i[a] && si[b] < si[a]);
            else take = si[b] != INT64_MAX &&
                        (si[a] == INT64_MAX || sv[b] < sv[a] || (sv[b] == sv[a] && si[b] < si[a]));
            if (take) {
                sv[a] = sv[b];
                sv_i[a] = sv_i[b];
                si[a] = si[b];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) best[0] = (int32_t)si[0];
}

__global__ void __launch_bounds__(1024) k_argmin(int64_t R, const int64_t *e_i64,
                                                 const double *e_f64, int32_t *best) {
    argmin_body(R, e_i64, e_f64, best);
}

__global__ void __launch_bounds__(1024) k_argmin_batch(const ScoreTask *__restrict__ tasks) {
    const ScoreTask &t = tasks[blockIdx.y];
    argmin_body(t.R, t.e_i64, t.e_f64, t.best);
}

inline unsigned grid1(int64_t total, int block, int64_t cap = 65536) {
    int64_t g = (total + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

template <typename F> hipError_t dispatch_q(int32_t dt, F &&f) {
    switch (dt) {
        case QPA_I8: return f((int8_t)0);
        case QPA_I16: return f((int16_t)0);
        case QPA_I32: return f((int32_t)0);
        case QPA_F32: return f(0.0f);
        default: return hipErrorInvalidValue;
    }
}

// One launch for small instances; above CANON_ROWS_PER_PART rows, P <= CANON_PARTS
// workgroups of rows and a single-workgroup reduction of their partials.
void canon_reduce(int64_t n, const double *row_abs, const double *row_max, const double *row_k,
                  double *parts, int32_t is_int, CanonScalars *sc, CanonScalars *mirror,
                  hipStream_t st) {
    if (n <= CANON_ROWS_PER_PART || parts == nullptr) {
        k_canon_finalize<<<1, 1024, 0, st>>>(n, row_abs, row_max, row_k, nullptr, is_int, sc,
                                             mirror);
        return;
    }
    int64_t P = (n + CANON_ROWS_PER_PART - 1) / CANON_ROWS_PER_PART;
    if (P > CANON_PARTS) P = CANON_PARTS;
    const int64_t rows = (n + P - 1) / P;
    k_canon_part<<<(unsigned)P, 1024, 0, st>>>(n, rows, row_abs, row_max, row_k, parts);
    k_canon_finalize<<<1, 1024, 0, st>>>(P, nullptr, nullptr, nullptr, parts, is_int, sc,
                                         mirror);
}

// Best state over the trajectory: workgroup r compares replica r's energy of the state
// after `t` steps with its best so far (the first sample is always taken; a tie keeps the
// earlier state) and, when lower, copies the state's spins, then the energy and step.
__global__ void __launch_bounds__(256) k_track_best(int64_t n, const double *__restrict__ energy,
                                                    const int8_t *__restrict__ spins, int32_t t,
                                                    int32_t first, double *__restrict__ best_e,
                                                    int32_t *__restrict__ best_t,
                                                    int8_t *__restrict__ best_s) {
    const int64_t r = blockIdx.x;
    const double e = energy[r];
    // one decision for the workgroup, taken before anything of the replica is written
    __shared__ int take;
    if (threadIdx.x == 0) take = first || e < best_e[r];
    __syncthreads();
    if (!take) return;
    const int8_t *src = spins + r * n;
    int8_t *dst = best_s + r * n;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
    if (threadIdx.x == 0) {
        best_e[r] = e;
        best_t[r] = t;
    }
}

}  // namespace

hipError_t launch_canon_dense(const qpa_problem &p, float *J_f32, uint16_t *Jb, int64_t npad,
                              float *b_f32, int64_t *b_i64, double *b_f64, double *row_abs,
                              double *row_max, double *row_k, double *parts, CanonScalars *sc,
                              hipStream_t st) {
    const int64_t n = p.n;
    const int32_t is_qubo = p.kind == QPA_KIND_QUBO;
    const int32_t is_int = dtype_is_int(p.coupling_dtype) &&
                           (p.linear == nullptr || dtype_is_int(p.linear_dtype));
    hipError_t e = hipMemsetAsync(sc, 0, sizeof(CanonScalars), st);
    if (e != hipSuccess) return e;
    e = dispatch_q(p.coupling_dtype, [&](auto tag) {
        using T = decltype(tag);
        const T *Q = static_cast<const T *>(p.dense);
        k_dense_rows<T><<<(unsigned)((n + 3) / 4), 256, 0, st>>>(
            n, Q, p.linear, p.linear_dtype, is_qubo, J_f32, b_f32, b_i64, b_f64, row_abs,
            row_max, row_k, sc);
        int64_t nb = (n + 31) / 32;
        k_dense_sym<T><<<dim3((unsigned)nb, (unsigned)nb), 256, 0, st>>>(n, Q, sc);
        canon_reduce(n, row_abs, row_max, row_k, parts, is_int, sc, nullptr, st);
        if (Jb) k_dense_bf16<T><<<grid1(npad * npad, 256), 256, 0, st>>>(n, npad, Q, sc, Jb);
        return hipGetLastError();
    });
    return e;
}

hipError_t launch_canon_csr(const qpa_problem &p, float *b_f32, int64_t *b_i64, double *b_f64,
                            double *row_abs, double *row_max, double *row_k, double *parts,
                            CanonScalars *sc, hipStream_t st, CanonScalars *mirror) {
    const int64_t n = p.n;
    const int32_t is_qubo = p.kind == QPA_KIND_QUBO;
    const int32_t is_int = dtype_is_int(p.coupling_dtype) &&
                           (p.linear == nullptr || dtype_is_int(p.linear_dtype));
    hipError_t e = hipMemsetAsync(sc, 0, sizeof(CanonScalars), st);
    if (e != hipSuccess) return e;
    auto run = [&](auto wtag, auto itag) {
        using TW = decltype(wtag);
        using TI = decltype(itag);
        if (csr_rows_by_wave(p) && !std::is_floating_point<TW>::value)
            k_csr_rows_wave<TW, TI><<<(unsigned)((n + 3) / 4), 256, 0, st>>>(
                n, p.nnz, p.row_ptr, static_cast<const TI *>(p.col),
                static_cast<const TW *>(p.weights), p.linear, p.linear_dtype, is_qubo, b_f32,
                b_i64, b_f64, row_abs, row_max, row_k, sc);
        else
            k_csr_rows<TW, TI><<<grid1(n, 256, INT64_MAX), 256, 0, st>>>(
                n, p.nnz, p.row_ptr, static_cast<const TI *>(p.col),
                static_cast<const TW *>(p.weights), p.linear, p.linear_dtype, is_qubo, b_f32,
                b_i64, b_f64, row_abs, row_max, row_k, sc);
        canon_reduce(n, row_abs, row_max, row_k, parts, is_int, sc, mirror, st);
        return hipGetLastError();
    };
    return dispatch_q(p.coupling_dtype, [&](auto wtag) {
        if (p.index_dtype == QPA_I16) return run(wtag, (int16_t)0);
        return run(wtag, (int32_t)0);
    });
}

hipError_t launch_init_state(int64_t n, int64_t R, uint64_t seed, float sigma0, float *x,
                             float *m, int64_t ld_r, int64_t ld_i, int64_t Rpad, int64_t npad,
                             hipStream_t st) {
    k_init_state<<<grid1(Rpad * npad, 256), 256, 0, st>>>(n, R, seed, sigma0, x, m, ld_r, ld_i,
                                                          Rpad, npad);
    return hipGetLastError();
}

hipError_t launch_canon_batch(const CanonTask *tasks, int32_t ntask, qpa_dtype coupling,
                              qpa_dtype index, int64_t max_n, hipStream_t st) {
    const int64_t gx = (max_n + 3) / 4;
    if (gx < 1 || gx > INT32_MAX) return hipErrorInvalidValue;
    auto run = [&](auto wtag, auto itag) {
        using TW = decltype(wtag);
        using TI = decltype(itag);
        for (int32_t c0 = 0; c0 < ntask; c0 += 65535) {
            const unsigned rows = (unsigned)std::min(65535, ntask - c0);
            k_canon_zero_batch<<<dim3(1, rows), 64, 0, st>>>(tasks + c0);
            k_csr_rows_wave_batch<TW, TI><<<dim3((unsigned)gx, rows), 256, 0, st>>>(tasks + c0);
            k_canon_finalize_batch<<<dim3(1, rows), 1024, 0, st>>>(tasks + c0);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    auto byw = [&](auto itag) -> hipError_t {
        switch (coupling) {
            case QPA_I8: return run((int8_t)0, itag);
            case QPA_I16: return run((int16_t)0, itag);
            case QPA_I32: return run((int32_t)0, itag);
            default: return hipErrorInvalidValue;
        }
    };
    return index == QPA_I16 ? byw((int16_t)0) : byw((int32_t)0);
}

hipError_t launch_slot_init_batch(const SlotInitTask *tasks, int32_t ntask, int64_t max_elems,
                                  float sigma0, hipStream_t st) {
    for (int32_t c0 = 0; c0 < ntask; c0 += 65535) {
        const dim3 g(grid1(max_elems, 256, 256), (unsigned)std::min(65535, ntask - c0));
        k_slot_init_batch<<<g, 256, 0, st>>>(tasks + c0, sigma0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_copy_state(int64_t n, int64_t R, const float *src, int64_t s_ld_r,
                             int64_t s_ld_i, float *dst, int64_t d_ld_r, int64_t d_ld_i,
                             hipStream_t st) {
    if (R * n == 0) return hipSuccess;
    k_copy_state<<<grid1(R * n, 256), 256, 0, st>>>(n, R, src, s_ld_r, s_ld_i, dst, d_ld_r,
                                                    d_ld_i);
    return hipGetLastError();
}

hipError_t launch_pad_f32(int64_t n, int64_t np, const float *src, float *dst, hipStream_t st) {
    if (np <= 0) return hipSuccess;
    k_pad_f32<<<grid1(np, 256), 256, 0, st>>>(n, np, src, dst);
    return hipGetLastError();
}

hipError_t launch_export_spins(int64_t n, int64_t R, const float *x, int64_t ld_r,
                               int64_t ld_i, int8_t *spins, hipStream_t st) {
    if (R * n == 0) return hipSuccess;
    k_export_spins<<<grid1(R * n, 256), 256, 0, st>>>(n, R, x, ld_r, ld_i, spins);
    return hipGetLastError();
}

// Integer CSR instances averaging 16 or more entries per row take the wave-per-row
// kernels.
bool csr_rows_by_wave(const qpa_problem &p) {
    const bool is_int = dtype_is_int(p.coupling_dtype) &&
                        (p.linear == nullptr || dtype_is_int(p.linear_dtype));
    return p.format == QPA_FMT_CSR && is_int && p.nnz >= 16 * p.n;
}

int64_t energy_partial_blocks(const qpa_problem &p) {
    if (p.format == QPA_FMT_DENSE) return (p.n + 15) / 16;
    if (csr_rows_by_wave(p)) return (p.n + 3) / 4;
    return (p.n + 255) / 256;
}

hipError_t launch_energy(const qpa_problem &p, const int64_t *b_i64, const double *b_f64,
                         const CanonScalars *sc, const int8_t *spins, int64_t R,
                         int64_t *e_i64, double *e_f64, double *partial, int64_t partial_len,
                         uint64_t *words, hipStream_t st) {
    const int64_t n = p.n;
    const int32_t is_qubo = p.kind == QPA_KIND_QUBO;
    const bool is_int = dtype_is_int(p.coupling_dtype) &&
                        (p.linear == nullptr || dtype_is_int(p.linear_dtype));
    const int64_t nblk = energy_partial_blocks(p);
    if (nblk * R > partial_len) return hipErrorInvalidValue;
    const unsigned gy = (unsigned)((R + ER - 1) / ER);
    hipError_t e;
    if (p.format == QPA_FMT_DENSE) {
        const int64_t nw = (n + 63) / 64;
        k_spin_rowbits<<<(unsigned)((R + 3) / 4), 256, 0, st>>>(n, R, nw, spins, words);
        e = dispatch_q(p.coupling_dtype, [&](auto tag) {
            using T = decltype(tag);
            const T *Q = static_cast<const T *>(p.dense);
            k_energy_dense<T><<<(unsigned)nblk, 1024, 0, st>>>(n, nw, Q, is_int ? b_i64 : nullptr,
                                                               b_f64, words, R, partial);
            return hipGetLastError();
        });
    } else {
        auto run = [&](auto wtag, auto itag) {
            using TW = decltype(wtag);
            using TI = decltype(itag);
            const TW *w = static_cast<const TW *>(p.weights);
            const TI *c = static_cast<const TI *>(p.col);
            if (csr_rows_by_wave(p))
                k_energy_csr_wave<TW, TI><<<dim3((unsigned)nblk, gy), 256, 0, st>>>(
                    n, p.row_ptr, c, w, b_i64, spins, R, partial);
            else if (is_int)
                k_energy_csr<TW, TI, true><<<dim3((unsigned)nblk, gy), 256, 0, st>>>(
                    n, p.row_ptr, c, w, b_i64, b_f64, spins, R, partial);
            else
                k_energy_csr<TW, TI, false><<<dim3((unsigned)nblk, gy), 256, 0, st>>>(
                    n, p.row_ptr, c, w, b_i64, b_f64, spins, R, partial);
            return hipGetLastError();
        };
        e = dispatch_q(p.coupling_dtype, [&](auto wtag) {
            if (p.index_dtype == QPA_I16) return run(wtag, (int16_t)0);
            return run(wtag, (int32_t)0);
        });
    }
    if (e != hipSuccess) return e;
    k_energy_finalize<<<grid1(R * 64, 256, INT64_MAX), 256, 0, st>>>(
        R, nblk, partial, is_int ? 1 : 0, is_qubo, p.format == QPA_FMT_DENSE ? 1 : 0, sc,
        is_int ? e_i64 : nullptr, e_f64);
    return hipGetLastError();
}

hipError_t launch_argmin(int64_t R, const int64_t *e_i64, const double *e_f64, int32_t *best,
                         hipStream_t st) {
    k_argmin<<<1, 1024, 0, st>>>(R, e_i64, e_f64, best);
    return hipGetLastError();
}

hipError_t launch_track_best(int64_t n, int64_t R, const double *energy, const int8_t *spins,
                             int32_t t, bool first, double *best_e, int32_t *best_t,
                             int8_t *best_s, hipStream_t st) {
    if (R < 1 || R > INT32_MAX || n < 1) return hipErrorInvalidValue;
    k_track_best<<<(unsigned)R, 256, 0, st>>>(n, energy, spins, t, first ? 1 : 0, best_e, best_t,
                                              best_s);
    return hipGetLastError();
}

// Batched scoring launches: instance y of the table in grid row y (at most 65535 rows a
// launch); every kernel returns from the blocks an instance does not need.
constexpr int32_t SCORE_ROWS = 65535;

hipError_t launch_export_spins_batch(const ScoreTask *tasks, int32_t ntask, int64_t max_elems,
                                     hipStream_t st) {
    for (int32_t c0 = 0; c0 < ntask; c0 += SCORE_ROWS) {
        const dim3 g(grid1(max_elems, 256, 64), (unsigned)std::min(SCORE_ROWS, ntask - c0));
        k_export_spins_batch<<<g, 256, 0, st>>>(tasks + c0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int64_t energy_bits_blocks(int64_t n) { return (n + EB_ROWS - 1) / EB_ROWS; }

hipError_t launch_energy_bits_batch(const ScoreTask *tasks, int32_t ntask, qpa_dtype coupling,
                                    qpa_dtype index, int64_t max_n, int64_t max_words,
                                    hipStream_t st) {
    if (max_n < 1 || max_n > EBITS_MAX_N) return hipErrorInvalidValue;
    auto run = [&](auto wtag, auto itag) {
        using TW = decltype(wtag);
        using TI = decltype(itag);
        for (int32_t c0 = 0; c0 < ntask; c0 += SCORE_ROWS) {
            const unsigned rows = (unsigned)std::min(SCORE_ROWS, ntask - c0);
            k_spin_words_batch<<<dim3(grid1(max_words * 64, 256, 1024), rows), 256, 0, st>>>(
                tasks + c0);
            k_energy_bits_batch<TW, TI>
                <<<dim3((unsigned)energy_bits_blocks(max_n), rows), 256, 0, st>>>(tasks + c0);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    auto byw = [&](auto itag) -> hipError_t {
        switch (coupling) {
            case QPA_I8: return run((int8_t)0, itag);
            case QPA_I16: return run((int16_t)0, itag);
            case QPA_I32: return run((int32_t)0, itag);
            default: return hipErrorInvalidValue;
        }
    };
    return index == QPA_I16 ? byw((int16_t)0) : byw((int32_t)0);
}

hipError_t launch_finalize_argmin_batch(const ScoreTask *tasks, int32_t ntask, int64_t max_R,
                                        hipStream_t st) {
    for (int32_t c0 = 0; c0 < ntask; c0 += SCORE_ROWS) {
        const unsigned rows = (unsigned)std::min(SCORE_ROWS, ntask - c0);
        k_energy_finalize_batch<<<dim3(grid1(max_R * 64, 256, INT64_MAX), rows), 256, 0, st>>>(
            tasks + c0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        k_argmin_batch<<<dim3(1, rows), 1024, 0, st>>>(tasks + c0);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace qpa
