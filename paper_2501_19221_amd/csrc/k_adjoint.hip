// Relaxed PA (analog spins in the target part, s := x) and its reverse-mode adjoint.
//
// Forward step t (FP32, each operation rounded separately):
//   f = J x_t;  g = lambda_t x_t + f + b;  m_{t+1} = alpha m_t - eta g;
//   y_{t+1} = x_t + m_{t+1};  x_{t+1} = clip(y_{t+1}, -1, 1).
// Loss: L = scale * sum_r [ (1/2) x_T^T J x_T + b^T x_T ]  (scale = 1/replicas for a mean).
// Reverse, with mu_{T+1} = 0 and xbar_T = scale (J x_T + b):
//   ybar = xbar_{t+1} * [|y_{t+1}| <= 1];   mu = ybar + alpha mu_next;
//   dL/deta += <mu, -g_t>,  dL/dalpha += <mu, m_t>,  dL/dlambda_t = <mu, -eta x_t>;
//   xbar_t = ybar - eta (lambda_t mu + J mu).
// State layout: [R][n] FP32, replica-major.  Products with J: dense couplings through an
// LDS-tiled FP32 kernel, CSR couplings through a row gather; both sum in ascending column
// order.  Inner products are accumulated per workgroup in double and written to a
// per-step partial table, reduced at the end in a fixed order (deterministic).
#include "qpa_internal.h"

namespace qpa {
namespace {

constexpr int TB = 64, TK = 32;

// out[r][i] = sum_k J[i][k] v[r][k]   (dense FP32 J, [n][n] row-major)
__global__ void __launch_bounds__(256) k_dense_apply(int64_t n, int64_t R,
                                                     const float *__restrict__ J,
                                                     const float *__restrict__ v,
                                                     float *__restrict__ out) {
    __shared__ float As[TK][TB + 1];
    __shared__ float Bs[TK][TB + 1];
    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;
    const int64_t r0 = (int64_t)blockIdx.y * TB, i0 = (int64_t)blockIdx.x * TB;
    float acc[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[q][c] = 0.0f;
    for (int64_t k0 = 0; k0 < n; k0 += TK) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            int idx = tid + e * 256;
            int row = idx / TK, kk = idx % TK;
            int64_t k = k0 + kk;
            int64_t r = r0 + row, i = i0 + row;
            As[kk][row] = (r < R && k < n) ? v[r * n + k] : 0.0f;
            Bs[kk][row] = (i < n && k < n) ? J[i * n + k] : 0.0f;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < TK; ++kk) {
            float a[4], bb[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = As[kk][4 * ty + q];
#pragma unroll
            for (int c = 0; c < 4; ++c) bb[c] = Bs[kk][tx + 16 * c];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[q][c] = __fadd_rn(acc[q][c], __fmul_rn(a[q], bb[c]));
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int64_t r = r0 + 4 * ty + q;
        if (r >= R) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            int64_t i = i0 + tx + 16 * c;
            if (i < n) out[r * n + i] = acc[q][c];
        }
    }
}

template <typename TW, typename TI>
__global__ void __launch_bounds__(256) k_csr_apply(int64_t n, int64_t R,
                                                   const int32_t *__restrict__ rp,
                                                   const TI *__restrict__ col,
                                                   const TW *__restrict__ w, int skip_diag,
                                                   const float *__restrict__ v,
                                                   float *__restrict__ out) {
    const int64_t total = R * n;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = q / n, i = q - r * n;
        const float *vr = v + r * n;
        float acc = 0.0f;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int64_t j = (int64_t)col[k];
            if (skip_diag && j == i) continue;
            acc = __fadd_rn(acc, __fmul_rn((float)w[k], vr[j]));
        }
        out[q] = acc;
    }
}

// forward update given f = J x (in place on x, m); optionally records y = x + m'.
__global__ void __launch_bounds__(256) k_rel_update(int64_t n, int64_t R, const float *__restrict__ f,
                                                    const float *__restrict__ b, float lam,
                                                    float eta, float alpha, float *__restrict__ x,
                                                    float *__restrict__ m) {
    const int64_t total = R * n;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q % n;
        const float xv = x[q];
        float g = __fadd_rn(__fadd_rn(__fmul_rn(lam, xv), f[q]), b[i]);
        float mn = __fsub_rn(__fmul_rn(alpha, m[q]), __fmul_rn(eta, g));
        float y = __fadd_rn(xv, mn);
        x[q] = fminf(1.0f, fmaxf(-1.0f, y));
        m[q] = mn;
    }
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh[k];
    return s;
}

// loss partial: sum (1/2) x f + b x; xbar = scale (f + b)
__global__ void __launch_bounds__(256) k_rel_loss(int64_t n, int64_t R, const float *__restrict__ x,
                                                  const float *__restrict__ f,
                                                  const float *__restrict__ b, double scale,
                                                  float *__restrict__ xbar,
                                                  double *__restrict__ part) {
    __shared__ double sh[4];
    const int64_t total = R * n;
    double acc = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q % n;
        const double xv = x[q], fv = f[q], bv = b[i];
        acc += 0.5 * xv * fv + bv * xv;
        xbar[q] = (float)(scale * (fv + bv));
    }
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s * scale;
}

// Reverse part A for step t: from the state (x_t, m_t) and f_t = J x_t, rebuild g_t,
// m_{t+1}, y_{t+1}; ybar = xbar * [|y| <= 1]; mu = ybar + alpha mu (in place);
// partial inner products <mu,-g>, <mu,m_t>, <mu,-eta x_t> for this block.
__global__ void __launch_bounds__(256) k_rel_rev_a(int64_t n, int64_t R,
                                                   const float *__restrict__ x,
                                                   const float *__restrict__ m,
                                                   const float *__restrict__ f,
                                                   const float *__restrict__ b, float lam,
                                                   float eta, float alpha,
                                                   float *__restrict__ xbar,
                                                   float *__restrict__ mu,
                                                   double *__restrict__ part /* [3][nblk] */) {
    __shared__ double sh[4];
    const int64_t total = R * n;
    double se = 0.0, sa = 0.0, sl = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q % n;
        const float xv = x[q], mv = m[q];
        float g = __fadd_rn(__fadd_rn(__fmul_rn(lam, xv), f[q]), b[i]);
        float mn = __fsub_rn(__fmul_rn(alpha, mv), __fmul_rn(eta, g));
        float y = __fadd_rn(xv, mn);
        const float yb = fabsf(y) <= 1.0f ? xbar[q] : 0.0f;
        const float u = __fadd_rn(yb, __fmul_rn(alpha, mu[q]));
        mu[q] = u;
        xbar[q] = yb;                                  // holds ybar until part B
        se += (double)u * (double)(-g);
        sa += (double)u * (double)mv;
        sl += (double)u * (double)(-eta * xv);
    }
    const double a = block_sum(se, sh);
    const double c = block_sum(sa, sh);
    const double d = block_sum(sl, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = a;
        part[gridDim.x + blockIdx.x] = c;
        part[2 * gridDim.x + blockIdx.x] = d;
    }
}

// Reverse part B: xbar_t = ybar - eta (lambda_t mu + J mu), with Jmu = J mu.
__global__ void __launch_bounds__(256) k_rel_rev_b(int64_t count, const float *__restrict__ mu,
                                                   const float *__restrict__ Jmu, float lam,
                                                   float eta, float *__restrict__ xbar) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count;
         q += (int64_t)gridDim.x * blockDim.x) {
        float inner = __fadd_rn(__fmul_rn(lam, mu[q]), Jmu[q]);
        xbar[q] = __fsub_rn(xbar[q], __fmul_rn(eta, inner));
    }
}

// final reduction of the per-step partial tables (fixed order)
__global__ void __launch_bounds__(256) k_rel_finish(int32_t T, int32_t nblk,
                                                    const double *__restrict__ part_steps,
                                                    const double *__restrict__ part_loss,
                                                    double *__restrict__ loss,
                                                    double *__restrict__ d_eta,
                                                    double *__restrict__ d_alpha,
                                                    double *__restrict__ d_lam) {
    for (int32_t t = threadIdx.x; t < T; t += blockDim.x) {
        const double *p = part_steps + (int64_t)t * 3 * nblk;
        double l = 0.0;
        for (int32_t k = 0; k < nblk; ++k) l += p[2 * nblk + k];
        d_lam[t] = l;
    }
    if (threadIdx.x == 0) {
        double e = 0.0, a = 0.0, L = 0.0;
        for (int32_t t = 0; t < T; ++t) {
            const double *p = part_steps + (int64_t)t * 3 * nblk;
            for (int32_t k = 0; k < nblk; ++k) {
                e += p[k];
                a += p[nblk + k];
            }
        }
        for (int32_t k = 0; k < nblk; ++k) L += part_loss[k];
        *loss = L;
        *d_eta = e;
        *d_alpha = a;
    }
}

}  // namespace

int32_t rel_blocks(int64_t count) {
    int64_t g = (count + 255) / 256;
    if (g > 1024) g = 1024;
    return (int32_t)(g < 1 ? 1 : g);
}

hipError_t launch_rel_apply(const qpa_problem &p, const float *Jf, bool skip_diag, int64_t R,
                            const float *v, float *out, hipStream_t st) {
    const int64_t n = p.n;
    if (p.format == QPA_FMT_DENSE) {
        dim3 grid((unsigned)((n + TB - 1) / TB), (unsigned)((R + TB - 1) / TB));
        k_dense_apply<<<grid, 256, 0, st>>>(n, R, Jf, v, out);
        return hipGetLastError();
    }
    const unsigned g = (unsigned)rel_blocks(R * n);
    auto run = [&](auto wtag, auto itag) {
        using TW = decltype(wtag);
        using TI = decltype(itag);
        k_csr_apply<TW, TI><<<g, 256, 0, st>>>(n, R, p.row_ptr, static_cast<const TI *>(p.col),
                                               static_cast<const TW *>(p.weights),
                                               skip_diag ? 1 : 0, v, out);
        return hipGetLastError();
    };
    auto byw = [&](auto itag) -> hipError_t {
        switch (p.coupling_dtype) {
            case QPA_I8: return run((int8_t)0, itag);
            case QPA_I16: return run((int16_t)0, itag);
            case QPA_I32: return run((int32_t)0, itag);
            default: return run(0.0f, itag);
        }
    };
    return p.index_dtype == QPA_I16 ? byw((int16_t)0) : byw((int32_t)0);
}

hipError_t launch_rel_update(int64_t n, int64_t R, const float *f, const float *b, float lam,
                             float eta, float alpha, float *x, float *m, hipStream_t st) {
    k_rel_update<<<rel_blocks(R * n), 256, 0, st>>>(n, R, f, b, lam, eta, alpha, x, m);
    return hipGetLastError();
}

hipError_t launch_rel_loss(int64_t n, int64_t R, const float *x, const float *f, const float *b,
                           double scale, float *xbar, double *part, hipStream_t st) {
    k_rel_loss<<<rel_blocks(R * n), 256, 0, st>>>(n, R, x, f, b, scale, xbar, part);
    return hipGetLastError();
}

hipError_t launch_rel_rev_a(int64_t n, int64_t R, const float *x, const float *m, const float *f,
                            const float *b, float lam, float eta, float alpha, float *xbar,
                            float *mu, double *part, hipStream_t st) {
    k_rel_rev_a<<<rel_blocks(R * n), 256, 0, st>>>(n, R, x, m, f, b, lam, eta, alpha, xbar, mu,
                                                   part);
    return hipGetLastError();
}

hipError_t launch_rel_rev_b(int64_t count, const float *mu, const float *Jmu, float lam,
                            float eta, float *xbar, hipStream_t st) {
    k_rel_rev_b<<<rel_blocks(count), 256, 0, st>>>(count, mu, Jmu, lam, eta, xbar);
    return hipGetLastError();
}

hipError_t launch_rel_finish(int32_t T, int32_t nblk, const double *part_steps,
                             const double *part_loss, double *loss, double *d_eta,
                             double *d_alpha, double *d_lam, hipStream_t st) {
    k_rel_finish<<<1, 256, 0, st>>>(T, nblk, part_steps, part_loss, loss, d_eta, d_alpha, d_lam);
    return hipGetLastError();
}

}  // namespace qpa
