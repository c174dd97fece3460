// Sparse (CSR) PA step (App. B): h_i = sum_k w_k s_{col_k} + b_i, then the fused update.
//
// Replicas are packed into groups of G lanes (G a power of two, G <= 64).  A wave handles
// V = 64/G consecutive variables x G replicas of one group, so every lane owns one
// (variable, replica) pair; the lanes of a variable read the same CSR entries (broadcast)
// and each picks its own replica's spin bit out of a shared 64-bit word.
// Layouts:
//   x, m   [np][Rp] FP32, replica fastest (Rp = groups * G)
//   spins  words[g][w], 64 bits each: variable i, replica r = g*G + rl sits in word
//          w = i / V at bit (i % V) * G + rl; bit set <=> spin -1.
// Integer couplings are summed in int32 (exact: rows are validated below 2^24) and the
// total converted once; float couplings are summed in FP32 in row order.  Both match the
// definition's ascending-entry order.
#include "qpa_internal.h"

namespace qpa {
namespace {

__device__ __forceinline__ void pa_update(float h, float lam, float eta, float alpha, float &x,
                                          float &m) {
    float g = __fadd_rn(__fmul_rn(lam, x), h);
    float mn = __fsub_rn(__fmul_rn(alpha, m), __fmul_rn(eta, g));
    float y = __fadd_rn(x, mn);
    y = fminf(1.0f, fmaxf(-1.0f, y));
    m = mn;
    x = y;
}

constexpr int CSR_BATCH = 4;   // row entries whose loads are issued together

template <typename TW, typename TI, bool INT>
__global__ void __launch_bounds__(256) k_csr_step(
    int64_t n, int64_t Rp, int G, int shiftG, int64_t nwords, const int32_t *__restrict__ rp,
    const TI *__restrict__ col, const TW *__restrict__ wts, int skip_diag,
    const float *__restrict__ b, const uint64_t *__restrict__ s_cur,
    uint64_t *__restrict__ s_nxt, float *__restrict__ x, float *__restrict__ m,
    float *__restrict__ h_last, int t, const float *__restrict__ lam, float eta, float alpha) {
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t g = blockIdx.y;
    const int V = 64 >> shiftG;
    const int vsub = lane >> shiftG, rl = lane & (G - 1);
    const int64_t i = w * V + vsub;
    const int64_t r = g * G + rl;
    const uint64_t *sg = s_cur + g * nwords;
    const int wsh = 6 - shiftG;
    bool neg = false;
    if (w < nwords && i < n) {
        // every load that does not depend on a gathered value is issued up front; the
        // entries of the row follow in batches of CSR_BATCH (column and weight loads, then
        // all spin-word gathers, then the sums in entry order), so a wave waits for three
        // memory round trips per batch instead of two per entry
        const int64_t gi = i * Rp + r;
        const int64_t k0 = rp[i], k1 = rp[i + 1];
        float xv = x[gi], mv = m[gi];
        const float bi = b[i];
        int32_t ai = 0;
        float af = 0.0f;
        auto batch = [&](int64_t kb) {
            int64_t j[CSR_BATCH];
            TW wk[CSR_BATCH];
            uint64_t word[CSR_BATCH];
#pragma unroll
            for (int d = 0; d < CSR_BATCH; ++d) {
                const int64_t k = kb + d < k1 ? kb + d : k1 - 1;   // in bounds: kb < k1
                j[d] = (int64_t)col[k];
                wk[d] = wts[k];
            }
#pragma unroll
            for (int d = 0; d < CSR_BATCH; ++d) {
                word[d] = 0;
                if (kb + d < k1) word[d] = sg[j[d] >> wsh];
            }
#pragma unroll
            for (int d = 0; d < CSR_BATCH; ++d) {
                if (kb + d >= k1 || (skip_diag && j[d] == i)) continue;
                const int bit = (int)((word[d] >> (((j[d] & (V - 1)) << shiftG) + rl)) & 1u);
                if (INT) {
                    const int32_t v = (int32_t)wk[d];
                    ai += bit ? -v : v;
                } else {
                    const float v = (float)wk[d];
                    af = __fadd_rn(af, bit ? -v : v);
                }
            }
        };
        if (k0 < k1) batch(k0);   // the first batch outside the loop: most rows end in it
        for (int64_t kb = k0 + CSR_BATCH; kb < k1; kb += CSR_BATCH) batch(kb);
        const float h = INT ? __fadd_rn((float)ai, bi) : __fadd_rn(af, bi);
        pa_update(h, lam[t], eta, alpha, xv, mv);
        x[gi] = xv;
        m[gi] = mv;
        if (h_last) h_last[gi] = h;
        neg = xv < 0.0f;
    }
    const uint64_t bal = __ballot(neg);
    if (lane == 0 && w < nwords) s_nxt[g * nwords + w] = bal;
}

__global__ void __launch_bounds__(256) k_csr_pack(int64_t n, int64_t Rp, int G, int shiftG,
                                                  int64_t nwords, const float *__restrict__ x,
                                                  uint64_t *__restrict__ sbits) {
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t g = blockIdx.y;
    const int V = 64 >> shiftG;
    const int64_t i = w * V + (lane >> shiftG);
    const int64_t r = g * G + (lane & (G - 1));
    bool neg = false;
    if (w < nwords && i < n) neg = x[i * Rp + r] < 0.0f;
    const uint64_t bal = __ballot(neg);
    if (lane == 0 && w < nwords) sbits[g * nwords + w] = bal;
}

int log2i(int v) {
    int s = 0;
    while ((1 << s) < v) ++s;
    return s;
}

}  // namespace

int csr_group_size(int64_t R) {
    int G = 1;
    while (G < R && G < 64) G <<= 1;
    return G;
}

int64_t csr_words_per_group(int64_t n, int G) {
    const int V = 64 / G;
    return (n + V - 1) / V;
}

hipError_t launch_csr_pack_spins(int64_t n, int64_t Rp, int G, const float *x, uint64_t *sbits,
                                 hipStream_t st) {
    const int64_t nwords = csr_words_per_group(n, G);
    dim3 grid((unsigned)((nwords + 3) / 4), (unsigned)(Rp / G));
    k_csr_pack<<<grid, 256, 0, st>>>(n, Rp, G, log2i(G), nwords, x, sbits);
    return hipGetLastError();
}

hipError_t launch_csr_step(const CsrView &c, int64_t Rp, int G, const float *b_f32,
                           const uint64_t *s_cur, uint64_t *s_nxt, float *x, float *m,
                           float *h_last, int32_t t, const float *lam, float eta, float alpha,
                           bool is_int, hipStream_t st) {
    const int64_t nwords = csr_words_per_group(c.n, G);
    dim3 grid((unsigned)((nwords + 3) / 4), (unsigned)(Rp / G));
    const int sh = log2i(G);
    auto run = [&](auto wtag, auto itag) {
        using TW = decltype(wtag);
        using TI = decltype(itag);
        const TW *w = static_cast<const TW *>(c.w);
        const TI *cl = static_cast<const TI *>(c.col);
        if (is_int)
            k_csr_step<TW, TI, true><<<grid, 256, 0, st>>>(c.n, Rp, G, sh, nwords, c.rp, cl, w,
                                                           c.skip_diag, b_f32, s_cur, s_nxt, x,
                                                           m, h_last, t, lam, eta, alpha);
        else
            k_csr_step<TW, TI, false><<<grid, 256, 0, st>>>(c.n, Rp, G, sh, nwords, c.rp, cl, w,
                                                            c.skip_diag, b_f32, s_cur, s_nxt, x,
                                                            m, h_last, t, lam, eta, alpha);
        return hipGetLastError();
    };
    auto byw = [&](auto itag) -> hipError_t {
        switch (c.w_dt) {
            case QPA_I8: return run((int8_t)0, itag);
            case QPA_I16: return run((int16_t)0, itag);
            case QPA_I32: return run((int32_t)0, itag);
            case QPA_F32: return run(0.0f, itag);
            default: return hipErrorInvalidValue;
        }
    };
    if (c.col_dt == QPA_I16) return byw((int16_t)0);
    return byw((int32_t)0);
}

}  // namespace qpa
