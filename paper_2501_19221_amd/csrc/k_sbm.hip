// Simulated Bifurcation Machine steps (App. B) and the power method that sets its c0.
//
// Hamilton's equations of the oscillator network, dq/dt = a0 p and
// dp/dt = -(q^2 + a0 - a(t)) q + c0 (J' q + h'), advanced by symplectic Euler with step
// dt: p from the positions of the step, then q from the new p.  The problem arrives in
// the minimisation convention of the PA path (canonical J, b), and the machine runs on
// (J', h') = (-J, -b), so its force is -c0 (J q + b).  Per element, FP32, one rounding
// per operation in this order:
//   g = (sum_j J_ij q_j, one fused multiply-add per term, ascending j) + b_i
//   w = ((q q + a0) - a) q;  F = -w - c0 g;  p = p + dt F;  q = q + (dt a0) p
//
// State layout: q, p [n][Rp] FP32, replica fastest.  Every step reads q_in and writes
// q_out (the update is synchronous), p in place.
//
// Dense couplings: an LDS-tiled FP32 product on the vector units.  A workgroup owns a
// 128 (replicas) x 128 (variables) output tile; each of its 256 threads holds 8 x 8
// sums and adds one term per reduction index with a fused multiply-add, in ascending
// order, so every sum is bit-identical to the sequential definition.  Chunks of 32
// reduction indices of q (from [n][Rp]: contiguous in replicas) and J (symmetric, so row
// k of J gives column k: contiguous in variables) are double-buffered in LDS; the next
// chunk is prefetched into registers while the current one is multiplied.  The update
// runs in the epilogue on the tile's 16384 elements.
//
// CSR couplings: one lane per (row, replica); the G lanes of a row (G = replicas per
// row group, a power of two <= 64) read the row's entries once per wave and gather
// q_in of the neighbours from [n][Rp] rows, contiguous in replicas.
//
// Power method (FP64): v_0 = 2u - 1 (u the top 24 bits of SplitMix64 output i + 1 of the
// seed), normalised; then iters times w = J v, v = w / ||w||; the estimate is ||J v||.
// Each product writes per-workgroup partial sums of w^2 and one small launch reduces
// them in a fixed order, so the result is deterministic.
#include "fp32_tiled.h"

namespace qpa {
namespace {

__device__ __forceinline__ void sbm_point(float f, float bi, float a, float a0, float c0,
                                          float dt, float adt, float &q, float &p, float &g) {
    g = __fadd_rn(f, bi);
    const float qq = __fmul_rn(q, q);
    const float w = __fmul_rn(__fsub_rn(__fadd_rn(qq, a0), a), q);
    const float cg = __fmul_rn(c0, g);
    const float force = __fsub_rn(-w, cg);
    const float pn = __fadd_rn(p, __fmul_rn(dt, force));
    p = pn;
    q = __fadd_rn(q, __fmul_rn(adt, pn));
}

// SBM epilogue: the symplectic step of every (variable, replica) of the tile.
struct SbmEpilogue {
    const float *b, *c0p;
    float a, a0, dt;
    const float *qi;
    float *qo, *p, *gout;
    // thread holds replicas r0 + 64h + 4ty + e (h, e < 2, 4) and variables
    // i0 + 64(v/4) + 4tx + v%4
    __device__ __forceinline__ void operator()(float (&acc)[8][8], int64_t n, int64_t Rp,
                                               int64_t i0, int64_t r0, int tx, int ty) const {
        const float c0 = *c0p;
        const float adt = __fmul_rn(dt, a0);
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int64_t i = i0 + 64 * (v >> 2) + 4 * tx + (v & 3);
            if (i >= n) continue;
            const float bi = b[i];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int64_t idx = i * Rp + r0 + 64 * h + 4 * ty;
                float4 qv = *reinterpret_cast<const float4 *>(qi + idx);
                float4 pv = *reinterpret_cast<const float4 *>(p + idx);
                float4 gv;
                sbm_point(acc[4 * h + 0][v], bi, a, a0, c0, dt, adt, qv.x, pv.x, gv.x);
                sbm_point(acc[4 * h + 1][v], bi, a, a0, c0, dt, adt, qv.y, pv.y, gv.y);
                sbm_point(acc[4 * h + 2][v], bi, a, a0, c0, dt, adt, qv.z, pv.z, gv.z);
                sbm_point(acc[4 * h + 3][v], bi, a, a0, c0, dt, adt, qv.w, pv.w, gv.w);
                *reinterpret_cast<float4 *>(qo + idx) = qv;
                *reinterpret_cast<float4 *>(p + idx) = pv;
                if (gout) *reinterpret_cast<float4 *>(gout + idx) = gv;
            }
        }
    }
};

__device__ __forceinline__ void pa_point(float acc, float bi, float lt, float eta, float alpha,
                                         float &x, float &m, float &s, float &h) {
    h = __fadd_rn(acc, bi);
    const float g = __fadd_rn(__fmul_rn(lt, x), h);
    const float mn = __fsub_rn(__fmul_rn(alpha, m), __fmul_rn(eta, g));
    x = fminf(1.0f, fmaxf(-1.0f, __fadd_rn(x, mn)));
    m = mn;
    s = x >= 0.0f ? 1.0f : -1.0f;
}

// PA epilogue (App. B): h = J s + b, the momentum update and clipping, and the next
// step's spins s' = sign(x') as +-1 floats.  With s = +-1 every product of the tiled sum
// is exact and a fused multiply-add rounds once, so the field equals the ascending sum.
struct PaEpilogue {
    const float *b, *lam;
    int t;
    float eta, alpha;
    float *x, *m, *s_nxt, *h_last;
    __device__ __forceinline__ void operator()(float (&acc)[8][8], int64_t n, int64_t Rp,
                                               int64_t i0, int64_t r0, int tx, int ty) const {
        const float lt = lam[t];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int64_t i = i0 + 64 * (v >> 2) + 4 * tx + (v & 3);
            if (i >= n) continue;
            const float bi = b[i];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int64_t idx = i * Rp + r0 + 64 * h + 4 * ty;
                float4 xv = *reinterpret_cast<const float4 *>(x + idx);
                float4 mv = *reinterpret_cast<const float4 *>(m + idx);
                float4 sv, hv;
                pa_point(acc[4 * h + 0][v], bi, lt, eta, alpha, xv.x, mv.x, sv.x, hv.x);
                pa_point(acc[4 * h + 1][v], bi, lt, eta, alpha, xv.y, mv.y, sv.y, hv.y);
                pa_point(acc[4 * h + 2][v], bi, lt, eta, alpha, xv.z, mv.z, sv.z, hv.z);
                pa_point(acc[4 * h + 3][v], bi, lt, eta, alpha, xv.w, mv.w, sv.w, hv.w);
                *reinterpret_cast<float4 *>(x + idx) = xv;
                *reinterpret_cast<float4 *>(m + idx) = mv;
                *reinterpret_cast<float4 *>(s_nxt + idx) = sv;
                if (h_last) *reinterpret_cast<float4 *>(h_last + idx) = hv;
            }
        }
    }
};


// CSR step: lane -> (row, replica).  Wave w covers replica chunk w % (Rp / G) and rows
// (w / (Rp / G)) * (64 / G) + lane / G.
constexpr int SBM_BATCH = 4;   // row entries whose loads are issued together

template <typename TW, typename TI>
__global__ void __launch_bounds__(256) k_sbm_csr_step(int64_t n, int64_t Rp, int G,
                                                      const int32_t *__restrict__ rp,
                                                      const TI *__restrict__ col,
                                                      const TW *__restrict__ w, int skip_diag,
                                                      const float *__restrict__ b,
                                                      const float *__restrict__ c0p, float a,
                                                      float a0, float dt,
                                                      const float *__restrict__ qi,
                                                      float *__restrict__ qo,
                                                      float *__restrict__ p,
                                                      float *__restrict__ gout) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t chunks = Rp / G;
    const int64_t chunk = wave % chunks;
    const int64_t row = (wave / chunks) * (64 / G) + lane / G;
    if (row >= n) return;
    const int64_t r = chunk * G + (lane & (G - 1));
    // loads that do not depend on a gathered value first, then the row in batches of
    // SBM_BATCH entries (columns and weights, then the gathers, then the fused
    // multiply-adds in entry order)
    const int32_t k0 = rp[row], k1 = rp[row + 1];
    const int64_t idx = row * Rp + r;
    float q = qi[idx], pv = p[idx], g;
    const float brow = b[row];
    float acc = 0.0f;
    auto batch = [&](int32_t kb) {
        int64_t j[SBM_BATCH];
        float wk[SBM_BATCH], qj[SBM_BATCH];
#pragma unroll
        for (int d = 0; d < SBM_BATCH; ++d) {
            const int32_t k = kb + d < k1 ? kb + d : k1 - 1;   // in bounds: kb < k1
            j[d] = (int64_t)col[k];
            wk[d] = (float)w[k];
        }
#pragma unroll
        for (int d = 0; d < SBM_BATCH; ++d) {
            qj[d] = 0.0f;
            if (kb + d < k1) qj[d] = qi[j[d] * Rp + r];
        }
#pragma unroll
        for (int d = 0; d < SBM_BATCH; ++d) {
            if (kb + d >= k1 || (skip_diag && j[d] == row)) continue;
            acc = __fmaf_rn(wk[d], qj[d], acc);
        }
    };
    if (k0 < k1) batch(k0);
    for (int32_t kb = k0 + SBM_BATCH; kb < k1; kb += SBM_BATCH) batch(kb);
    sbm_point(acc, brow, a, a0, *c0p, dt, __fmul_rn(dt, a0), q, pv, g);
    qo[idx] = q;
    p[idx] = pv;
    if (gout) gout[idx] = g;
}

// Resident CSR steps: one launch runs every step.  A workgroup owns G replicas and every
// variable; thread t owns variables t, t + 1024, ... (VPT of them) and keeps their q, p in
// registers for all steps.  The CSR structure (row pointers int32, columns uint16,
// weights FP32) and the positions of the G replicas ([n][G] FP32) live in LDS.  A step
// computes every owned field from LDS (one fused multiply-add per entry and replica, in
// row order, as the streamed kernel), a barrier, the update and the new positions into
// LDS, a barrier.  a(t) comes from a table the host fills with the same FP32 expression
// as the per-step launches.
constexpr int SRT = 1024;

// the G positions of variable j (row j of the [n][G] LDS array)
template <int G>
__device__ __forceinline__ void sbm_lds_read(const float *qv, int32_t j, float (&out)[G]) {
    if constexpr (G == 8) {
        const float4 lo = reinterpret_cast<const float4 *>(qv)[2 * j];
        const float4 hi = reinterpret_cast<const float4 *>(qv)[2 * j + 1];
        out[0] = lo.x; out[1] = lo.y; out[2] = lo.z; out[3] = lo.w;
        out[4] = hi.x; out[5] = hi.y; out[6] = hi.z; out[7] = hi.w;
    } else if constexpr (G == 4) {
        const float4 v = reinterpret_cast<const float4 *>(qv)[j];
        out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    } else if constexpr (G == 2) {
        const float2 v = reinterpret_cast<const float2 *>(qv)[j];
        out[0] = v.x; out[1] = v.y;
    } else {
        out[0] = qv[j];
    }
}

template <int G, int VPT>
__global__ void __launch_bounds__(SRT) k_sbm_csr_resident(
    int32_t n, int32_t nnz, int64_t R, int64_t Rp, const int32_t *__restrict__ rp_g,
    const void *__restrict__ col_g, int32_t col_dt, const void *__restrict__ w_g, int32_t w_dt,
    int32_t skip_diag, const float *__restrict__ b, const float *__restrict__ c0p,
    const float *__restrict__ atab, float a0, float dt, float *__restrict__ q,
    float *__restrict__ p, float *__restrict__ gout, int32_t t0, int32_t t1) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    int32_t *rp = reinterpret_cast<int32_t *>(lds);
    float *wf = reinterpret_cast<float *>(rp + (n + 1));
    uint16_t *col = reinterpret_cast<uint16_t *>(wf + nnz);
    const size_t qoff = ((size_t)(n + 1) * 4 + (size_t)nnz * 6 + 15) & ~(size_t)15;
    float *qv = reinterpret_cast<float *>(lds + qoff);
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * G;

    for (int32_t k = tid; k <= n; k += SRT) rp[k] = rp_g[k];
    for (int32_t k = tid; k < nnz; k += SRT) {
        col[k] = (uint16_t)(col_dt == QPA_I16 ? (int32_t) static_cast<const int16_t *>(col_g)[k]
                                              : static_cast<const int32_t *>(col_g)[k]);
        switch (w_dt) {
            case QPA_I8: wf[k] = (float)static_cast<const int8_t *>(w_g)[k]; break;
            case QPA_I16: wf[k] = (float)static_cast<const int16_t *>(w_g)[k]; break;
            case QPA_I32: wf[k] = (float)static_cast<const int32_t *>(w_g)[k]; break;
            default: wf[k] = static_cast<const float *>(w_g)[k]; break;
        }
    }
    float qs[VPT][G], ps[VPT][G], gs[VPT][G], bi[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int32_t i = tid + u * SRT;
        bi[u] = 0.0f;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            qs[u][g] = 0.0f;
            ps[u][g] = 0.0f;
            gs[u][g] = 0.0f;
        }
        if (i < n) {
            bi[u] = b[i];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (r0 + g < R) {
                    qs[u][g] = q[(int64_t)i * Rp + r0 + g];
                    ps[u][g] = p[(int64_t)i * Rp + r0 + g];
                }
                qv[i * G + g] = qs[u][g];
            }
        }
    }
    if (tid < G) qv[n * G + tid] = 0.0f;       // row n: the +0.0 of unused cache slots
    const float c0 = *c0p;
    const float adt = __fmul_rn(dt, a0);
    __syncthreads();
    // the first CACHE off-diagonal entries of each owned row in registers; the step issues
    // their position reads together.  Unused slots carry weight -0.0 and read row n of the
    // positions, which holds +0.0: the product is exactly -0.0, and adding -0.0 leaves
    // every value unchanged (also -0.0, which a product w q that underflows can leave)
    // at most 32 cached positions and, with 8 variables per thread, one entry per row
    constexpr int CA = VPT >= 8 ? 1 : (16 / VPT) < 8 ? (16 / VPT) : 8;
    constexpr int CACHE = CA * G > 32 ? 32 / G : CA;
    int32_t cj[VPT][CACHE], crest[VPT];
    float cw[VPT][CACHE];
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int32_t i = tid + u * SRT;
        int32_t k = 0, k1 = 0, cnt = 0;
        if (i < n) {
            k = rp[i];
            k1 = rp[i + 1];
        }
#pragma unroll
        for (int c = 0; c < CACHE; ++c) {
            cj[u][c] = n;
            cw[u][c] = -0.0f;
        }
        for (; k < k1 && cnt < CACHE; ++k) {
            const int32_t j = col[k];
            if (skip_diag && j == i) continue;
#pragma unroll
            for (int c = 0; c < CACHE; ++c)
                if (c == cnt) {
                    cj[u][c] = j;
                    cw[u][c] = wf[k];
                }
            ++cnt;
        }
        crest[u] = k;
    }
    for (int32_t t = t0; t < t1; ++t) {
        const float a = atab[t];
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            const int32_t i = tid + u * SRT;
            float acc[G];
#pragma unroll
            for (int g = 0; g < G; ++g) acc[g] = 0.0f;
            if (i < n) {
                float qc[CACHE][G];
#pragma unroll
                for (int c = 0; c < CACHE; ++c) sbm_lds_read<G>(qv, cj[u][c], qc[c]);
#pragma unroll
                for (int c = 0; c < CACHE; ++c)
#pragma unroll
                    for (int g = 0; g < G; ++g) acc[g] = __fmaf_rn(cw[u][c], qc[c][g], acc[g]);
                const int32_t k1 = rp[i + 1];
                for (int32_t k = crest[u]; k < k1; ++k) {
                    const int32_t j = col[k];
                    if (skip_diag && j == i) continue;
                    const float w = wf[k];
                    float qj[G];
                    sbm_lds_read<G>(qv, j, qj);
#pragma unroll
                    for (int g = 0; g < G; ++g) acc[g] = __fmaf_rn(w, qj[g], acc[g]);
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g) gs[u][g] = acc[g];
        }
        __syncthreads();                    // every read of this step's positions is done
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            const int32_t i = tid + u * SRT;
            if (i < n) {
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    float gv;
                    sbm_point(gs[u][g], bi[u], a, a0, c0, dt, adt, qs[u][g], ps[u][g], gv);
                    gs[u][g] = gv;
                    qv[i * G + g] = qs[u][g];
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int32_t i = tid + u * SRT;
        if (i >= n) continue;
#pragma unroll
        for (int g = 0; g < G; ++g)
            if (r0 + g < R) {
                q[(int64_t)i * Rp + r0 + g] = qs[u][g];
                p[(int64_t)i * Rp + r0 + g] = ps[u][g];
                if (gout && t1 > t0) gout[(int64_t)i * Rp + r0 + g] = gs[u][g];
            }
    }
}

__global__ void k_set_f32(float *dst, float v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = v;
}

// ------------------------------------------------------------------ power method
__device__ __forceinline__ uint64_t pw_splitmix(uint64_t seed, uint64_t k) {
    uint64_t z = seed + k * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// sum over the workgroup (256 threads); result valid in thread 0
__device__ __forceinline__ double group_sum(double v, double *sh) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return s;
}

__global__ void __launch_bounds__(256) k_pw_start(int64_t n, uint64_t seed,
                                                  double *__restrict__ v,
                                                  double *__restrict__ part) {
    __shared__ double sh[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double x = 0.0;
    if (i < n) {
        const uint64_t top = pw_splitmix(seed, (uint64_t)i + 1u) >> 40;
        x = 2.0 * (double)top / 16777216.0 - 1.0;
        v[i] = x;
    }
    const double s = group_sum(x * x, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// w_i = inv * sum_j J_ij v_j with one wave per row (dense, caller's dtype, QUBO diagonal
// skipped); part[block] = sum of w_i^2 over the block's 4 rows.
template <typename T>
__global__ void __launch_bounds__(256) k_pw_dense(int64_t n, const T *__restrict__ Q,
                                                  int skip_diag, const double *__restrict__ v,
                                                  const double *__restrict__ nrm,
                                                  double *__restrict__ w,
                                                  double *__restrict__ part) {
    __shared__ double sh[4];
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    double s = 0.0;
    if (row < n) {
        const T *qr = Q + row * n;
        for (int64_t j = lane; j < n; j += 64)
            if (!(skip_diag && j == row)) s += (double)qr[j] * v[j];
    }
    s = wave_sum(s);
    double y = 0.0;
    if (row < n) {
        y = s * nrm[1];
        if (lane == 0) w[row] = y;
    }
    const double tot = group_sum(lane == 0 ? y * y : 0.0, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// The same for CSR couplings, one thread per row.
template <typename TW, typename TI>
__global__ void __launch_bounds__(256) k_pw_csr(int64_t n, const int32_t *__restrict__ rp,
                                                const TI *__restrict__ col,
                                                const TW *__restrict__ wt, int skip_diag,
                                                const double *__restrict__ v,
                                                const double *__restrict__ nrm,
                                                double *__restrict__ w,
                                                double *__restrict__ part) {
    __shared__ double sh[4];
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double y = 0.0;
    if (row < n) {
        double s = 0.0;
        for (int32_t k = rp[row]; k < rp[row + 1]; ++k) {
            const int64_t j = (int64_t)col[k];
            if (!(skip_diag && j == row)) s += (double)wt[k] * v[j];
        }
        y = s * nrm[1];
        w[row] = y;
    }
    const double tot = group_sum(y * y, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// nrm[0] = sqrt(sum part), nrm[1] = 1 / nrm[0]; optionally rho = nrm[0] and
// c0 = (float)(1 / nrm[0]).
__global__ void __launch_bounds__(256) k_pw_finish(int64_t nb, const double *__restrict__ part,
                                                   double *__restrict__ nrm,
                                                   double *__restrict__ rho,
                                                   float *__restrict__ c0) {
    __shared__ double sh[4];
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < nb; k += 256) s += part[k];
    s = group_sum(s, sh);
    if (threadIdx.x == 0) {
        const double r = sqrt(s);
        nrm[0] = r;
        nrm[1] = r > 0.0 ? 1.0 / r : 0.0;
        if (rho) rho[0] = r;
        if (c0) c0[0] = r > 0.0 ? (float)(1.0 / r) : 0.0f;
    }
}

template <typename F>
hipError_t by_dtypes(const qpa_problem &p, F &&f) {
    auto byw = [&](auto itag) -> hipError_t {
        switch (p.coupling_dtype) {
            case QPA_I8: return f((int8_t)0, itag);
            case QPA_I16: return f((int16_t)0, itag);
            case QPA_I32: return f((int32_t)0, itag);
            default: return f(0.0f, itag);
        }
    };
    return p.index_dtype == QPA_I16 ? byw((int16_t)0) : byw((int32_t)0);
}

}  // namespace

int sbm_csr_group(int64_t R) {
    int G = 1;
    while (G < 64 && G < R) G <<= 1;
    return G;
}

int64_t sbm_rpad(const qpa_problem &p, int64_t R) {
    if (p.format == QPA_FMT_DENSE) return (R + SB_BR - 1) / SB_BR * SB_BR;
    const int G = sbm_csr_group(R);
    return (R + G - 1) / G * G;
}

int64_t dense_fp32_rpad(int64_t R) { return (R + SB_BR - 1) / SB_BR * SB_BR; }

hipError_t launch_dense_fp32_step(int64_t n, int64_t Rp, const float *J, const float *b,
                                  const float *s_cur, float *s_nxt, float *x, float *m,
                                  float *h_last, int32_t t, const float *lam, float eta,
                                  float alpha, hipStream_t st) {
    if (Rp % SB_BR || n < 1) return hipErrorInvalidValue;
    dim3 grid((unsigned)((n + SB_BI - 1) / SB_BI), (unsigned)(Rp / SB_BR));
    const PaEpilogue epi{b, lam, t, eta, alpha, x, m, s_nxt, h_last};
    if (n % 4 == 0)
        k_fp32_tiled_step<true, PaEpilogue><<<grid, 256, 0, st>>>(n, Rp, J, s_cur, epi);
    else
        k_fp32_tiled_step<false, PaEpilogue><<<grid, 256, 0, st>>>(n, Rp, J, s_cur, epi);
    return hipGetLastError();
}

int64_t pw_blocks(const qpa_problem &p) {
    const int64_t a = (p.n + 255) / 256;
    const int64_t d = p.format == QPA_FMT_DENSE ? (p.n + 3) / 4 : a;
    return a > d ? a : d;
}

hipError_t launch_sbm_step(const qpa_problem &p, const float *Jf, int64_t Rp, const float *b,
                           const float *c0p, float a, float a0, float dt, const float *q_in,
                           float *q_out, float *pm, float *g_out, hipStream_t st) {
    const int64_t n = p.n;
    if (p.format == QPA_FMT_DENSE) {
        dim3 grid((unsigned)((n + SB_BI - 1) / SB_BI), (unsigned)(Rp / SB_BR));
        const SbmEpilogue epi{b, c0p, a, a0, dt, q_in, q_out, pm, g_out};
        if (n % 4 == 0)
            k_fp32_tiled_step<true, SbmEpilogue><<<grid, 256, 0, st>>>(n, Rp, Jf, q_in, epi);
        else
            k_fp32_tiled_step<false, SbmEpilogue><<<grid, 256, 0, st>>>(n, Rp, Jf, q_in, epi);
        return hipGetLastError();
    }
    const int G = sbm_csr_group(Rp);
    const int64_t waves = ((n + (64 / G) - 1) / (64 / G)) * (Rp / G);
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    const int skip = p.kind == QPA_KIND_QUBO ? 1 : 0;
    return by_dtypes(p, [&](auto wtag, auto itag) {
        using TW = decltype(wtag);
        using TI = decltype(itag);
        k_sbm_csr_step<TW, TI><<<blocks, 256, 0, st>>>(
            n, Rp, G, p.row_ptr, static_cast<const TI *>(p.col),
            static_cast<const TW *>(p.weights), skip, b, c0p, a, a0, dt, q_in, q_out, pm, g_out);
        return hipGetLastError();
    });
}

size_t sbm_resident_lds(int64_t n, int64_t nnz, int G) {
    // positions of rows 0 .. n (row n: zeros for unused cache slots)
    return (((size_t)(n + 1) * 4 + (size_t)nnz * 6 + 15) & ~(size_t)15) +
           (size_t)(n + 1) * G * 4;
}

static int sbm_vpt(int64_t n) {
    const int64_t v = (n + SRT - 1) / SRT;
    return v <= 1 ? 1 : v <= 2 ? 2 : v <= 4 ? 4 : v <= 8 ? 8 : 0;
}

int sbm_resident_group(const qpa_problem &p, int64_t R, int cus) {
    if (p.format != QPA_FMT_CSR || p.n < 1 || p.n > RES_MAX_N || p.nnz > INT32_MAX) return 0;
    const int v = sbm_vpt(p.n);
    if (v == 0) return 0;
    for (int G = 8; G >= 1; G >>= 1) {
        if (v * G > 16 || sbm_resident_lds(p.n, p.nnz, G) > RES_MAX_LDS) continue;
        if (G > 1 && (R + G - 1) / G < cus) continue;
        return G;
    }
    return 0;
}

template <int G, int VPT>
static hipError_t launch_sbm_res_gv(const qpa_problem &pr, int64_t R, int64_t Rp, const float *b,
                                    const float *c0p, const float *atab, float a0, float dt,
                                    float *q, float *pm, float *g_out, int32_t t0, int32_t t1,
                                    hipStream_t st) {
    const size_t lds = sbm_resident_lds(pr.n, pr.nnz, G);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sbm_csr_resident<G, VPT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipGetLastError();
    const unsigned blocks = (unsigned)((R + G - 1) / G);
    k_sbm_csr_resident<G, VPT><<<blocks, SRT, lds, st>>>(
        (int32_t)pr.n, (int32_t)pr.nnz, R, Rp, pr.row_ptr, pr.col, pr.index_dtype, pr.weights,
        pr.coupling_dtype, pr.kind == QPA_KIND_QUBO ? 1 : 0, b, c0p, atab, a0, dt, q, pm, g_out,
        t0, t1);
    return hipGetLastError();
}

hipError_t launch_sbm_resident(const qpa_problem &pr, int G, int64_t R, int64_t Rp,
                               const float *b, const float *c0p, const float *atab, float a0,
                               float dt, float *q, float *pm, float *g_out, int32_t t0,
                               int32_t t1, hipStream_t st) {
    if (t1 <= t0) return hipSuccess;
    const int v = sbm_vpt(pr.n);
    if (v == 0 || v * G > 16 || sbm_resident_lds(pr.n, pr.nnz, G) > RES_MAX_LDS)
        return hipErrorInvalidValue;
#define QPA_SBM_RES(GG, VV)                                                                   \
    if (G == GG && v == VV)                                                                   \
        return launch_sbm_res_gv<GG, VV>(pr, R, Rp, b, c0p, atab, a0, dt, q, pm, g_out, t0, t1, \
                                         st);
    QPA_SBM_RES(8, 1)
    QPA_SBM_RES(8, 2)
    QPA_SBM_RES(4, 1)
    QPA_SBM_RES(4, 2)
    QPA_SBM_RES(4, 4)
    QPA_SBM_RES(2, 1)
    QPA_SBM_RES(2, 2)
    QPA_SBM_RES(2, 4)
    QPA_SBM_RES(2, 8)
    QPA_SBM_RES(1, 1)
    QPA_SBM_RES(1, 2)
    QPA_SBM_RES(1, 4)
    QPA_SBM_RES(1, 8)
#undef QPA_SBM_RES
    return hipErrorInvalidValue;
}

hipError_t launch_set_f32(float *dst, float v, hipStream_t st) {
    k_set_f32<<<1, 64, 0, st>>>(dst, v);
    return hipGetLastError();
}

hipError_t launch_power_method(const qpa_problem &p, int32_t iters, uint64_t seed, double *v,
                               double *w, double *part, double *nrm, double *rho, float *c0,
                               hipStream_t st) {
    const int64_t n = p.n;
    const int skip = p.kind == QPA_KIND_QUBO ? 1 : 0;
    const unsigned nb0 = (unsigned)((n + 255) / 256);
    k_pw_start<<<nb0, 256, 0, st>>>(n, seed, v, part);
    k_pw_finish<<<1, 256, 0, st>>>(nb0, part, nrm, nullptr, nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int32_t it = 0; it <= iters; ++it) {
        const bool last = it == iters;
        unsigned nb;
        if (p.format == QPA_FMT_DENSE) {
            nb = (unsigned)((n + 3) / 4);
            auto run = [&](auto tag) {
                using T = decltype(tag);
                k_pw_dense<T><<<nb, 256, 0, st>>>(n, static_cast<const T *>(p.dense), skip, v,
                                                  nrm, w, part);
                return hipGetLastError();
            };
            switch (p.coupling_dtype) {
                case QPA_I8: e = run((int8_t)0); break;
                case QPA_I16: e = run((int16_t)0); break;
                case QPA_I32: e = run((int32_t)0); break;
                default: e = run(0.0f); break;
            }
        } else {
            nb = nb0;
            e = by_dtypes(p, [&](auto wtag, auto itag) {
                using TW = decltype(wtag);
                using TI = decltype(itag);
                k_pw_csr<TW, TI><<<nb, 256, 0, st>>>(n, p.row_ptr,
                                                     static_cast<const TI *>(p.col),
                                                     static_cast<const TW *>(p.weights), skip,
                                                     v, nrm, w, part);
                return hipGetLastError();
            });
        }
        if (e != hipSuccess) return e;
        k_pw_finish<<<1, 256, 0, st>>>(nb, part, nrm, last ? rho : nullptr,
                                       last ? c0 : nullptr);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        double *tmp = v;
        v = w;
        w = tmp;
    }
    return hipSuccess;
}

}  // namespace qpa
