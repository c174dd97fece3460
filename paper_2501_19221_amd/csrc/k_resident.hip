// Sparse PA steps (App. B) with the whole state on chip: one launch runs every step.
//
// A workgroup owns G replicas (G in {1, 2, 4, 8}) and every variable of the instance.
// Thread t owns variables t, t + 1024, ... (VPT of them) for its workgroup's G replicas,
// and keeps their x and m in registers for all steps.  The instance's CSR structure is
// copied once into LDS (row pointers int32, columns uint16, weights int32 or FP32), next
// to two byte arrays of spins: byte j holds in bit g the sign of variable j in replica g
// of the workgroup (bit set <=> spin -1).  A step is, for every owned variable, a walk of
// its row -- one spin byte serves all G replicas -- followed by the fused update and one
// byte store; a workgroup barrier separates the steps.  The first CACHE off-diagonal
// entries of each owned row (CACHE = min(8, 16 / VPT)) are held in registers, so that a
// step issues their spin-byte reads together; longer rows continue from LDS in order.  Nothing is written to
// memory until the last step, when x and m go back to the workspace state ([n][Rp],
// replica fastest) and, if asked, the last field.
// The field sums follow the entry order of the row: int32 (exact; rows are validated
// below 2^24) for integer couplings, FP32 for float couplings, as in the streamed kernel.
// Integer rows whose sum of |w| stays below 2^16 (SW) take a packed form instead: with
// b' = b XOR [w < 0] a term is w (1 - 2b) = |w| (1 - 2b'), so the field is
// sum |w| - 2 A with A = sum |w| b' < 2^16.  The A of two replicas share one 32-bit word
// (16-bit lanes), summed modulo 2^32 as a row constant sum_{w<0} |w| (1 + 2^16) plus, per
// entry, w times the spread spin bits (bit of the first replica at 0, second at 16, from
// a 256-entry LDS table indexed by the spin byte): one signed 24-bit multiply-add per
// entry and replica pair.  The total is A_0 + 2^16 A_1 exactly, whatever the signs of the
// partial sums.  The cached entries are padded with zero weights, so the integer walk has
// no per-entry branch.
#include "qpa_internal.h"

namespace qpa {
namespace {

constexpr int RT = 1024;                 // threads per workgroup

__device__ __forceinline__ void pa_update(float h, float lam, float eta, float alpha, float &x,
                                          float &m) {
    float g = __fadd_rn(__fmul_rn(lam, x), h);
    float mn = __fsub_rn(__fmul_rn(alpha, m), __fmul_rn(eta, g));
    float y = __fadd_rn(x, mn);
    y = fminf(1.0f, fmaxf(-1.0f, y));
    m = mn;
    x = y;
}

template <typename T> __device__ __forceinline__ T ld_as(const void *p, int32_t dt, int64_t k) {
    switch (dt) {
        case QPA_I8: return (T) static_cast<const int8_t *>(p)[k];
        case QPA_I16: return (T) static_cast<const int16_t *>(p)[k];
        case QPA_I32: return (T) static_cast<const int32_t *>(p)[k];
        default: return (T) static_cast<const float *>(p)[k];
    }
}

// Spread words of spin byte b (NP of them) from the LDS table.
template <int NP>
__device__ __forceinline__ void lut_read(const uint32_t *lut, uint32_t b, uint32_t (&sp)[NP]) {
    if constexpr (NP == 4) {
        const uint4 v = reinterpret_cast<const uint4 *>(lut)[b];
        sp[0] = v.x; sp[1] = v.y; sp[2] = v.z; sp[3] = v.w;
    } else if constexpr (NP == 2) {
        const uint2 v = reinterpret_cast<const uint2 *>(lut)[b];
        sp[0] = v.x; sp[1] = v.y;
    } else {
        sp[0] = lut[b];
    }
}

constexpr size_t RES_LUT_BYTES = 256 * 4 * sizeof(uint32_t);

// LDS: spread table [256][4] uint32 | rp [n+1] int32 | w [nnz] int32 or float |
//      col [nnz] uint16 | spins [2][n] bytes
template <int G, int VPT, bool INT, bool SW>
__global__ void __launch_bounds__(RT) k_csr_resident(
    int32_t n, int32_t nnz, int64_t R, int64_t Rp, const int32_t *__restrict__ rp_g,
    const void *__restrict__ col_g, int32_t col_dt, const void *__restrict__ w_g, int32_t w_dt,
    int32_t skip_diag, const float *__restrict__ b, float *__restrict__ x,
    float *__restrict__ m, float *__restrict__ h_last, int32_t t0, int32_t t1,
    const float *__restrict__ lam, float eta, float alpha) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    uint32_t *lut = reinterpret_cast<uint32_t *>(lds);
    int32_t *rp = reinterpret_cast<int32_t *>(lds + RES_LUT_BYTES);
    int32_t *wi = rp + (n + 1);
    float *wf = reinterpret_cast<float *>(wi);
    uint16_t *col = reinterpret_cast<uint16_t *>(wi + nnz);
    uint8_t *sp0 = reinterpret_cast<uint8_t *>(col + nnz);
    uint8_t *sp1 = sp0 + n;
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * G;

    constexpr int NP = (G + 1) / 2;     // replica pairs, one 32-bit word each (SW)
    if (SW)
        for (int e = tid; e < 256 * NP; e += RT) {
            const uint32_t byte = (uint32_t)(e / NP), p = (uint32_t)(e % NP);
            lut[e] = ((byte >> (2 * p)) & 1u) | (((byte >> (2 * p + 1)) & 1u) << 16);
        }
    for (int32_t k = tid; k <= n; k += RT) rp[k] = rp_g[k];
    for (int32_t k = tid; k < nnz; k += RT) {
        col[k] = (uint16_t)(col_dt == QPA_I16 ? (int32_t) static_cast<const int16_t *>(col_g)[k]
                                              : static_cast<const int32_t *>(col_g)[k]);
        if (INT) wi[k] = ld_as<int32_t>(w_g, w_dt, k);
        else wf[k] = ld_as<float>(w_g, w_dt, k);
    }

    constexpr int CACHE = (16 / VPT) < 8 ? (16 / VPT) : 8;
    // cached entries of each owned row (diagonal entries of a QUBO left out), then the
    // LDS position where the rest of the row continues
    int32_t cj[VPT][CACHE];
    int32_t cwi[VPT][CACHE];
    float cwf[VPT][CACHE];
    int32_t ccount[VPT], crest[VPT];
    int32_t wabs[VPT];            // SW: sum of |w| over the row (diagonal excluded)
    uint32_t cneg[VPT];           // SW: sum over w < 0 of |w| (1 + 2^16), modulo 2^32
    float xs[VPT][G], ms[VPT][G], bi[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int32_t i = tid + u * RT;
        uint32_t byte = 0;
        bi[u] = 0.0f;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            xs[u][g] = 0.0f;
            ms[u][g] = 0.0f;
        }
        if (i < n) {
            bi[u] = b[i];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (r0 + g < R) {
                    xs[u][g] = x[(int64_t)i * Rp + r0 + g];
                    ms[u][g] = m[(int64_t)i * Rp + r0 + g];
                }
                byte |= (xs[u][g] < 0.0f ? 1u : 0u) << g;
            }
            sp0[i] = (uint8_t)byte;
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int32_t i = tid + u * RT;
        int32_t cnt = 0, k = 0, k1 = 0;
        if (i < n) {
            k = rp[i];
            k1 = rp[i + 1];
        }
#pragma unroll
        for (int c = 0; c < CACHE; ++c) {
            cj[u][c] = 0;
            cwi[u][c] = 0;
            cwf[u][c] = 0.0f;
        }
        wabs[u] = 0;
        cneg[u] = 0u;
        if (SW)
            for (int32_t kk = k; kk < k1; ++kk)
                if (!(skip_diag && col[kk] == i)) {
                    const int32_t a = wi[kk] < 0 ? -wi[kk] : wi[kk];
                    wabs[u] += a;
                    if (wi[kk] < 0) cneg[u] += (uint32_t)a * 0x10001u;
                }
        // take entries in row order until CACHE of them are held
        for (; k < k1 && cnt < CACHE; ++k) {
            const int32_t j = col[k];
            if (skip_diag && j == i) continue;
#pragma unroll
            for (int c = 0; c < CACHE; ++c)
                if (c == cnt) {
                    cj[u][c] = j;
                    if (INT) {
                        cwi[u][c] = wi[k];
                    } else {
                        cwf[u][c] = wf[k];
                    }
                }
            ++cnt;
        }
        ccount[u] = cnt;
        crest[u] = k;
    }

    uint8_t *cur = sp0, *nxt = sp1;
    for (int32_t t = t0; t < t1; ++t) {
        const float lt = lam[t];
        const bool last = (t == t1 - 1);
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            const int32_t i = tid + u * RT;
            if (i >= n) continue;
            int32_t ai[G];
            float af[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                ai[g] = 0;
                af[g] = 0.0f;
            }
            if (SW) {
                uint32_t acc[NP];
#pragma unroll
                for (int p = 0; p < NP; ++p) acc[p] = cneg[u];
                uint32_t cb[CACHE];
#pragma unroll
                for (int c = 0; c < CACHE; ++c) cb[c] = cur[cj[u][c]];
#pragma unroll
                for (int c = 0; c < CACHE; ++c) {
                    uint32_t sp[NP];
                    lut_read<NP>(lut, cb[c], sp);
#pragma unroll
                    for (int p = 0; p < NP; ++p)
                        acc[p] += (uint32_t)__mul24(cwi[u][c], (int32_t)sp[p]);
                }
                const int32_t k1 = rp[i + 1];
                for (int32_t k = crest[u]; k < k1; ++k) {
                    const int32_t j = col[k];
                    if (skip_diag && j == i) continue;
                    uint32_t sp[NP];
                    lut_read<NP>(lut, cur[j], sp);
#pragma unroll
                    for (int p = 0; p < NP; ++p) acc[p] += (uint32_t)__mul24(wi[k], (int32_t)sp[p]);
                }
#pragma unroll
                for (int g = 0; g < G; ++g)
                    ai[g] = wabs[u] - 2 * (int32_t)((acc[g >> 1] >> (16 * (g & 1))) & 0xffffu);
            } else {
            // cached entries: their spin bytes are read together, then summed in order
            uint32_t cb[CACHE];
#pragma unroll
            for (int c = 0; c < CACHE; ++c) cb[c] = c < ccount[u] ? cur[cj[u][c]] : 0u;
#pragma unroll
            for (int c = 0; c < CACHE; ++c) {
                if (c < ccount[u]) {
                    if (INT) {
                        const int32_t wk = cwi[u][c];
#pragma unroll
                        for (int g = 0; g < G; ++g) ai[g] += ((cb[c] >> g) & 1u) ? -wk : wk;
                    } else {
                        const float wk = cwf[u][c];
#pragma unroll
                        for (int g = 0; g < G; ++g)
                            af[g] = __fadd_rn(af[g], ((cb[c] >> g) & 1u) ? -wk : wk);
                    }
                }
            }
            const int32_t k1 = rp[i + 1];
            for (int32_t k = crest[u]; k < k1; ++k) {
                const int32_t j = col[k];
                if (skip_diag && j == i) continue;
                const uint32_t byte = cur[j];
                if (INT) {
                    const int32_t wk = wi[k];
#pragma unroll
                    for (int g = 0; g < G; ++g) ai[g] += ((byte >> g) & 1u) ? -wk : wk;
                } else {
                    const float wk = wf[k];
#pragma unroll
                    for (int g = 0; g < G; ++g)
                        af[g] = __fadd_rn(af[g], ((byte >> g) & 1u) ? -wk : wk);
                }
            }
            }
            uint32_t byte = 0;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const float h = INT ? __fadd_rn((float)ai[g], bi[u]) : __fadd_rn(af[g], bi[u]);
                pa_update(h, lt, eta, alpha, xs[u][g], ms[u][g]);
                byte |= (xs[u][g] < 0.0f ? 1u : 0u) << g;
                if (last && h_last && r0 + g < R) h_last[(int64_t)i * Rp + r0 + g] = h;
            }
            nxt[i] = (uint8_t)byte;
        }
        __syncthreads();
        uint8_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }

#pragma unroll
    for (int u = 0; u < VPT; ++u) {
        const int32_t i = tid + u * RT;
        if (i >= n) continue;
#pragma unroll
        for (int g = 0; g < G; ++g)
            if (r0 + g < R) {
                x[(int64_t)i * Rp + r0 + g] = xs[u][g];
                m[(int64_t)i * Rp + r0 + g] = ms[u][g];
            }
    }
}

template <int G, int VPT, bool INT, bool SW>
hipError_t launch_one(const CsrView &c, int64_t R, int64_t Rp, const float *b, float *x,
                      float *m, float *h_last, int32_t t0, int32_t t1, const float *lam,
                      float eta, float alpha, size_t lds, hipStream_t st) {
    const unsigned blocks = (unsigned)((R + G - 1) / G);
    // allow more than the default dynamic LDS; a runtime without the attribute leaves the
    // launch to report a real limit
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_csr_resident<G, VPT, INT, SW>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipGetLastError();
    k_csr_resident<G, VPT, INT, SW><<<blocks, RT, lds, st>>>(
        (int32_t)c.n, (int32_t)c.nnz, R, Rp, c.rp, c.col, c.col_dt, c.w, c.w_dt,
        c.skip_diag ? 1 : 0, b, x, m, h_last, t0, t1, lam, eta, alpha);
    return hipGetLastError();
}

template <int G, int VPT>
hipError_t launch_g_v(const CsrView &c, int64_t R, int64_t Rp, bool is_int, bool small_w,
                      const float *b, float *x, float *m, float *h_last, int32_t t0, int32_t t1,
                      const float *lam, float eta, float alpha, size_t lds, hipStream_t st) {
    if (is_int && small_w)
        return launch_one<G, VPT, true, true>(c, R, Rp, b, x, m, h_last, t0, t1, lam, eta,
                                              alpha, lds, st);
    if (is_int)
        return launch_one<G, VPT, true, false>(c, R, Rp, b, x, m, h_last, t0, t1, lam, eta,
                                               alpha, lds, st);
    return launch_one<G, VPT, false, false>(c, R, Rp, b, x, m, h_last, t0, t1, lam, eta, alpha,
                                            lds, st);
}

}  // namespace

size_t csr_resident_lds(int64_t n, int64_t nnz) {
    return RES_LUT_BYTES + sizeof(int32_t) * (size_t)(n + 1) +
           (sizeof(int32_t) + sizeof(uint16_t)) * (size_t)nnz + 2 * (size_t)n + 16;
}

namespace {
// variables per thread as instantiated: 1, 2, 4 or 8
int64_t resident_vpt(int64_t n) {
    const int64_t v = (n + RT - 1) / RT;
    return v <= 1 ? 1 : v <= 2 ? 2 : v <= 4 ? 4 : 8;
}
}  // namespace

int csr_resident_group(int64_t n, int64_t R, int cus) {
    if (n < 1 || n > RES_MAX_N) return 0;
    const int64_t v = resident_vpt(n);
    // the largest group that still gives every compute unit a workgroup, with at most
    // 16 (variable, replica) pairs per thread
    int G = 8;
    while (G > 1 && ((R + G - 1) / G < cus || v * G > 16)) G >>= 1;
    return v * G <= 16 ? G : 0;
}

hipError_t launch_csr_resident(const CsrView &c, int G, int64_t R, int64_t Rp, bool is_int,
                               bool small_w, const float *b, float *x, float *m, float *h_last,
                               int32_t t0, int32_t t1, const float *lam, float eta, float alpha,
                               hipStream_t st) {
    if (t1 <= t0) return hipSuccess;
    const size_t lds = csr_resident_lds(c.n, c.nnz);
    if (lds > RES_MAX_LDS || c.n > RES_MAX_N || c.nnz > INT32_MAX) return hipErrorInvalidValue;
    const int v = (int)resident_vpt(c.n);
    if (v * G > 16) return hipErrorInvalidValue;
#define QPA_RES_CASE(GG, VV)                                                                   \
    if (G == GG && v == VV)                                                                    \
        return launch_g_v<GG, VV>(c, R, Rp, is_int, small_w, b, x, m, h_last, t0, t1, lam, eta, \
                                  alpha, lds, st);
    QPA_RES_CASE(8, 1)
    QPA_RES_CASE(8, 2)
    QPA_RES_CASE(4, 1)
    QPA_RES_CASE(4, 2)
    QPA_RES_CASE(4, 4)
    QPA_RES_CASE(2, 1)
    QPA_RES_CASE(2, 2)
    QPA_RES_CASE(2, 4)
    QPA_RES_CASE(2, 8)
    QPA_RES_CASE(1, 1)
    QPA_RES_CASE(1, 2)
    QPA_RES_CASE(1, 4)
    QPA_RES_CASE(1, 8)
#undef QPA_RES_CASE
    return hipErrorInvalidValue;
}

}  // namespace qpa
