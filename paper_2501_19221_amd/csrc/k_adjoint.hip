// Relaxed PA (analog spins in the target part, s := x) and its reverse-mode adjoint, for
// one instance or a batch of instances sharing the dynamics parameters.
//
// Forward step t of one element (FP32, each operation rounded separately):
//   f = (J x_t)_i;  h = f + b_i;  g = lambda_t x + h;  m' = alpha m - eta g;
//   y = x + m';  x' = clip(y, -1, 1).
// Loss: L = scale * sum over instances and replicas of [ (1/2) x_T^T J x_T + b^T x_T ].
// Reverse, with mu_{T+1} = 0 and xbar_T = scale (J x_T + b):
//   A(t):  ybar = xbar_{t+1} * [|y_{t+1}| <= 1];  mu_{t+1} = ybar + alpha mu_{t+2};
//          dL/deta += <mu, -g_t>,  dL/dalpha += <mu, m_t>,  dL/dlambda_t = <mu, -eta x_t>
//   B(t):  xbar_t = ybar - eta (lambda_t mu_{t+1} + J mu_{t+1})
// A needs only the element's own values; B needs J mu, a product over neighbours.  A step
// of the reverse pass is one launch that runs B(t) and then A(t-1) on each element ("BA"),
// with mu double-buffered since neighbours read it; a segment's first step runs A alone
// and its last B alone, because the state of the step before a segment is recomputed
// only with the next segment.
//
// State: every vector is [rows][Rp] FP32 (replica fastest); instance k of a batch owns the
// global rows [row0_k, row0_k + n_k).  Replicas r >= R are padding: held at zero and left
// out of every sum.
// Products with J: CSR couplings through a gather (a wave = one row and 64 replicas, lane
// = replica, the row's entries fetched 64 at a time and walked in order, loads of four
// entries issued together); dense FP32 couplings through the LDS-tiled product shared with
// the SBM step, with the element work in its epilogue.  Both add one fused multiply-add
// per term in ascending column order.
// Inner products are accumulated in FP64 per thread, reduced per workgroup in a fixed
// order and written to a per-step table of partial sums, which one last launch reduces in
// a fixed order: results do not depend on the checkpoint interval or on timing.
#include "fp32_tiled.h"

namespace qpa {
namespace {

constexpr int REL_FWD = REL_MODE_FWD, REL_LOSS = REL_MODE_LOSS, REL_A = REL_MODE_A,
              REL_B = REL_MODE_B, REL_BA = REL_MODE_BA;

__device__ __forceinline__ void rel_fwd_point(float f, float bi, float lt, float eta,
                                              float alpha, float &x, float &m) {
    const float h = __fadd_rn(f, bi);
    const float g = __fadd_rn(__fmul_rn(lt, x), h);
    const float mn = __fsub_rn(__fmul_rn(alpha, m), __fmul_rn(eta, g));
    x = fminf(1.0f, fmaxf(-1.0f, __fadd_rn(x, mn)));
    m = mn;
}

// A(t) on one element from its stored state (x_t, m_t, f_t): the same FP32 operations as
// the forward step rebuild g_t and y_{t+1}.
__device__ __forceinline__ void rel_a_point(float x, float m, float f, float bi, float lt,
                                            float eta, float alpha, float xbar_next,
                                            float mu_next2, float &mu, float &yb, double &se,
                                            double &sa, double &sl) {
    const float h = __fadd_rn(f, bi);
    const float g = __fadd_rn(__fmul_rn(lt, x), h);
    const float mn = __fsub_rn(__fmul_rn(alpha, m), __fmul_rn(eta, g));
    const float y = __fadd_rn(x, mn);
    yb = fabsf(y) <= 1.0f ? xbar_next : 0.0f;
    mu = __fadd_rn(yb, __fmul_rn(alpha, mu_next2));
    se += (double)mu * (double)(-g);
    sa += (double)mu * (double)m;
    sl += (double)mu * (-(double)eta * (double)x);
}

__device__ __forceinline__ float rel_b_point(float yb, float mu, float jmu, float lt, float eta) {
    return __fsub_rn(yb, __fmul_rn(eta, __fadd_rn(__fmul_rn(lt, mu), jmu)));
}

__device__ __forceinline__ double rel_wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Fixed-order sum over the workgroup's waves (nw of them), result in thread 0.
__device__ __forceinline__ double rel_group_sum(double v, double *sh, int nw) {
    v = rel_wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < nw; ++k) s += sh[k];
    return s;
}

// Element work of one launch; `acc` is the product (J v)_i when the mode has one.
template <int MODE>
__device__ __forceinline__ void rel_element(const RelArgs &a, int64_t idx, bool live, float acc,
                                            float bi, double &s0, double &s1, double &s2) {
    if (MODE == REL_FWD) {
        float x = 0.0f, m = 0.0f;
        if (live) {
            x = a.xi[idx];
            m = a.mi[idx];
            rel_fwd_point(acc, bi, a.lam[a.t_f], a.eta, a.alpha, x, m);
        }
        a.xo[idx] = x;
        a.mo[idx] = m;
        if (a.fo) a.fo[idx] = live ? acc : 0.0f;
    } else if (MODE == REL_LOSS) {
        float xb = 0.0f;
        if (live) {
            const double x = a.xi[idx], f = acc, b = bi;
            s0 += 0.5 * x * f + b * x;
            xb = (float)(a.scale * (f + b));
        }
        a.xbar[idx] = xb;
    } else {
        float xbar_next = 0.0f;
        if (MODE == REL_A) {
            xbar_next = a.xbar[idx];
        } else {
            // B of the previous launch's step: xbar_t from ybar, mu_{t+1} and J mu_{t+1}
            const float xb = live ? rel_b_point(a.yb[idx], a.mu_in[idx], acc, a.lam[a.t_f],
                                                a.eta)
                                  : 0.0f;
            if (MODE == REL_B) {
                a.xbar[idx] = xb;
                return;
            }
            xbar_next = xb;
        }
        float mu = 0.0f, yb = 0.0f;
        if (live)
            rel_a_point(a.sx[idx], a.sm[idx], a.sf[idx], bi, a.lam[a.t_a], a.eta, a.alpha,
                        xbar_next, a.mu_in[idx], mu, yb, s0, s1, s2);
        a.mu_out[idx] = mu;
        a.yb[idx] = yb;
    }
}

// Writes this workgroup's partial sums (thread 0 holds the group sums).
template <int MODE>
__device__ __forceinline__ void rel_write_partials(const RelArgs &a, int64_t wg, double s0,
                                                   double s1, double s2, double *sh, int nw) {
    if (MODE == REL_FWD || MODE == REL_B) return;
    const double g0 = rel_group_sum(s0, sh, nw);
    if (MODE == REL_LOSS) {
        if (threadIdx.x == 0) a.part[a.slot0 + wg] = g0 * a.scale;
        return;
    }
    const double g1 = rel_group_sum(s1, sh, nw);
    const double g2 = rel_group_sum(s2, sh, nw);
    if (threadIdx.x == 0) {
        a.part[a.slot0 + wg] = g0;
        a.part[a.nblk + a.slot0 + wg] = g1;
        a.part[2 * a.nblk + a.slot0 + wg] = g2;
    }
}

template <typename T> __device__ __forceinline__ float as_weight(T w) { return (float)w; }

// Batched CSR launch (and, with MODE = REL_A, the element-wise pass over the rows of every
// instance).  Work item q = (row, 64-replica chunk); waves stride over the items in a
// fixed order.  The instance of a row is found by binary search over item0.
template <int MODE, typename TW, typename TI>
__global__ void __launch_bounds__(256) k_rel_rows(const RelInst *__restrict__ insts,
                                                  int32_t ninst, int64_t items, int32_t C,
                                                  const RelArgs a) {
    __shared__ double sh[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr bool GATHER = MODE != REL_A;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    const int64_t total = items * C;
    for (int64_t q = (int64_t)blockIdx.x * 4 + wv; q < total; q += (int64_t)gridDim.x * 4) {
        const int64_t item = q / C;
        const int c = (int)(q - item * C);
        int lo = 0, hi = ninst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (insts[mid].item0 <= item) lo = mid;
            else hi = mid - 1;
        }
        const RelInst &I = insts[lo];
        const int64_t i = item - I.item0;
        const int64_t r = (int64_t)c * 64 + lane;
        const int64_t idx = (I.row0 + i) * a.Rp + r;
        const bool live = r < a.R;
        float acc = 0.0f;
        if (GATHER) {
            const float *v = (MODE == REL_FWD || MODE == REL_LOSS) ? a.xi : a.mu_in;
            const float *vb = v + I.row0 * a.Rp + r;
            const TI *col = static_cast<const TI *>(I.col);
            const TW *w = static_cast<const TW *>(I.w);
            const int32_t k0 = I.rp[i], k1 = I.rp[i + 1];
            for (int32_t kb = k0; kb < k1; kb += 64) {
                int32_t jj = (int32_t)i;
                float ww = 0.0f;
                if (kb + lane < k1) {
                    jj = (int32_t)col[kb + lane];
                    ww = as_weight(w[kb + lane]);
                    // a stored QUBO diagonal is folded into b: weight 0 adds exactly nothing
                    if (I.skip_diag && jj == (int32_t)i) ww = 0.0f;
                }
                const int cnt = min(64, k1 - kb);
                int e = 0;
                for (; e + 4 <= cnt; e += 4) {
                    const int64_t j0 = __builtin_amdgcn_readlane(jj, e);
                    const int64_t j1 = __builtin_amdgcn_readlane(jj, e + 1);
                    const int64_t j2 = __builtin_amdgcn_readlane(jj, e + 2);
                    const int64_t j3 = __builtin_amdgcn_readlane(jj, e + 3);
                    const float v0 = vb[j0 * a.Rp], v1 = vb[j1 * a.Rp];
                    const float v2 = vb[j2 * a.Rp], v3 = vb[j3 * a.Rp];
                    const float w0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ww), e));
                    const float w1 =
                        __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ww), e + 1));
                    const float w2 =
                        __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ww), e + 2));
                    const float w3 =
                        __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ww), e + 3));
                    acc = __fmaf_rn(w0, v0, acc);
                    acc = __fmaf_rn(w1, v1, acc);
                    acc = __fmaf_rn(w2, v2, acc);
                    acc = __fmaf_rn(w3, v3, acc);
                }
                for (; e < cnt; ++e) {
                    const int64_t j = __builtin_amdgcn_readlane(jj, e);
                    const float we = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ww), e));
                    acc = __fmaf_rn(we, vb[j * a.Rp], acc);
                }
            }
        }
        rel_element<MODE>(a, idx, live, acc, I.b[i], s0, s1, s2);
    }
    rel_write_partials<MODE>(a, blockIdx.x, s0, s1, s2, sh, 4);
}

// Epilogue of the dense tiled product for every mode (b, and the state pointers in `a`,
// already offset to the instance's rows).
template <int MODE>
struct RelTileEpilogue {
    RelArgs a;
    const float *b;
    __device__ __forceinline__ void operator()(float (&acc)[8][8], int64_t n, int64_t Rp,
                                               int64_t i0, int64_t r0, int tx, int ty) const {
        __shared__ double sh[4];
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int64_t i = i0 + 64 * (v >> 2) + 4 * tx + (v & 3);
            if (i >= n) continue;
            const float bi = b[i];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t r = r0 + 64 * h + 4 * ty + e;
                    rel_element<MODE>(a, i * Rp + r, r < a.R, acc[4 * h + e][v], bi, s0, s1,
                                      s2);
                }
        }
        rel_write_partials<MODE>(a, (int64_t)blockIdx.y * gridDim.x + blockIdx.x, s0, s1, s2,
                                 sh, 4);
    }
};

__global__ void __launch_bounds__(256) k_rel_fill(double *__restrict__ p, int64_t count) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count;
         q += (int64_t)gridDim.x * blockDim.x)
        p[q] = 0.0;
}

// Final reduction of the per-step partial tables, in a fixed order: thread t sums the
// slots of steps t, t + 256, ... (d_lambda_t, and the step's d_eta and d_alpha terms,
// which it leaves in the step's first slots), then thread 0 sums the steps in order.
__global__ void __launch_bounds__(256) k_rel_finish(int32_t T, int32_t nblk,
                                                    double *__restrict__ part_steps,
                                                    const double *__restrict__ part_loss,
                                                    double *__restrict__ loss,
                                                    double *__restrict__ d_eta,
                                                    double *__restrict__ d_alpha,
                                                    double *__restrict__ d_lam) {
    const bool grads = d_eta || d_alpha || d_lam;
    if (grads)
        for (int32_t t = threadIdx.x; t < T; t += blockDim.x) {
            double *p = part_steps + (int64_t)t * 3 * nblk;
            double e = 0.0, a = 0.0, l = 0.0;
            for (int32_t k = 0; k < nblk; ++k) {
                e += p[k];
                a += p[nblk + k];
                l += p[2 * nblk + k];
            }
            p[0] = e;
            p[nblk] = a;
            if (d_lam) d_lam[t] = l;
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        double L = 0.0;
        for (int32_t k = 0; k < nblk; ++k) L += part_loss[k];
        *loss = L;
        if (grads) {
            double e = 0.0, a = 0.0;
            for (int32_t t = 0; t < T; ++t) {
                e += part_steps[(int64_t)t * 3 * nblk];
                a += part_steps[(int64_t)t * 3 * nblk + nblk];
            }
            if (d_eta) *d_eta = e;
            if (d_alpha) *d_alpha = a;
        }
    }
}

template <typename F>
hipError_t rel_by_dtypes(int32_t wdt, int32_t idt, F &&f) {
    auto byw = [&](auto itag) -> hipError_t {
        switch (wdt) {
            case QPA_I8: return f((int8_t)0, itag);
            case QPA_I16: return f((int16_t)0, itag);
            case QPA_I32: return f((int32_t)0, itag);
            default: return f(0.0f, itag);
        }
    };
    return idt == QPA_I16 ? byw((int16_t)0) : byw((int32_t)0);
}

template <int MODE>
hipError_t rel_rows_launch(const RelInst *insts, int32_t ninst, int64_t items, int32_t C,
                           int32_t wdt, int32_t idt, const RelArgs &a, hipStream_t st) {
    const unsigned g = (unsigned)rel_row_blocks(items, C);
    if (MODE == REL_A) {
        k_rel_rows<REL_A, float, int32_t><<<g, 256, 0, st>>>(insts, ninst, items, C, a);
        return hipGetLastError();
    }
    return rel_by_dtypes(wdt, idt, [&](auto wtag, auto itag) {
        using TW = decltype(wtag);
        using TI = decltype(itag);
        k_rel_rows<MODE, TW, TI><<<g, 256, 0, st>>>(insts, ninst, items, C, a);
        return hipGetLastError();
    });
}

template <int MODE>
hipError_t rel_tile_launch(int64_t n, const float *J, const float *b, const RelArgs &a,
                           hipStream_t st) {
    if (a.Rp % SB_BR || n < 1) return hipErrorInvalidValue;
    dim3 grid((unsigned)((n + SB_BI - 1) / SB_BI), (unsigned)(a.Rp / SB_BR));
    const RelTileEpilogue<MODE> epi{a, b};
    const float *q = (MODE == REL_FWD || MODE == REL_LOSS) ? a.xi : a.mu_in;
    if (n % 4 == 0)
        k_fp32_tiled_step<true, RelTileEpilogue<MODE>><<<grid, 256, 0, st>>>(n, a.Rp, J, q, epi);
    else
        k_fp32_tiled_step<false, RelTileEpilogue<MODE>><<<grid, 256, 0, st>>>(n, a.Rp, J, q, epi);
    return hipGetLastError();
}

}  // namespace

int64_t rel_row_blocks(int64_t items, int32_t C) {
    const int64_t waves = items * (int64_t)C;
    int64_t g = (waves + 3) / 4;
    if (g > REL_ROW_BLOCKS_MAX) g = REL_ROW_BLOCKS_MAX;
    return g < 1 ? 1 : g;
}

int64_t rel_tile_blocks(int64_t n, int64_t Rp) {
    return ((n + SB_BI - 1) / SB_BI) * (Rp / SB_BR);
}

hipError_t launch_rel_rows(int32_t mode, const RelInst *insts, int32_t ninst, int64_t items,
                           int32_t C, int32_t wdt, int32_t idt, const RelArgs &a,
                           hipStream_t st) {
    switch (mode) {
        case REL_FWD: return rel_rows_launch<REL_FWD>(insts, ninst, items, C, wdt, idt, a, st);
        case REL_LOSS: return rel_rows_launch<REL_LOSS>(insts, ninst, items, C, wdt, idt, a, st);
        case REL_A: return rel_rows_launch<REL_A>(insts, ninst, items, C, wdt, idt, a, st);
        case REL_B: return rel_rows_launch<REL_B>(insts, ninst, items, C, wdt, idt, a, st);
        case REL_BA: return rel_rows_launch<REL_BA>(insts, ninst, items, C, wdt, idt, a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_rel_tiles(int32_t mode, int64_t n, const float *J, const float *b,
                            const RelArgs &a, hipStream_t st) {
    switch (mode) {
        case REL_FWD: return rel_tile_launch<REL_FWD>(n, J, b, a, st);
        case REL_LOSS: return rel_tile_launch<REL_LOSS>(n, J, b, a, st);
        case REL_B: return rel_tile_launch<REL_B>(n, J, b, a, st);
        case REL_BA: return rel_tile_launch<REL_BA>(n, J, b, a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_rel_fill(double *p, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t g = (count + 255) / 256;
    if (g > 1024) g = 1024;
    k_rel_fill<<<(unsigned)g, 256, 0, st>>>(p, count);
    return hipGetLastError();
}

hipError_t launch_rel_finish(int32_t T, int32_t nblk, double *part_steps,
                             const double *part_loss, double *loss, double *d_eta,
                             double *d_alpha, double *d_lam, hipStream_t st) {
    k_rel_finish<<<1, 256, 0, st>>>(T, nblk, part_steps, part_loss, loss, d_eta, d_alpha, d_lam);
    return hipGetLastError();
}

}  // namespace qpa
