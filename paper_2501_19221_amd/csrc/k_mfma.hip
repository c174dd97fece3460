// Dense PA step on the CDNA4 matrix cores with BF16 couplings (App. B field J s + b,
// couplings stored as bf16(J / 2^e), FP32 accumulation, result scaled back by 2^e).
//
// One launch advances every replica by one step.  Output tile: 128 replicas x 128
// variables per workgroup (4 waves; wave w owns replicas 32w .. 32w+31 of the tile and all
// 128 variables, i.e. four 32x32 accumulators).  The reduction dimension walks in chunks
// of 64:
//   * the 128 x 64 block of J (bf16) is staged global -> registers -> LDS, double
//     buffered, rows padded to 144 bytes so that the 16-byte fragment reads of 8
//     consecutive lanes fall in distinct banks;
//   * the spins of the wave's 32 replicas arrive as one 64-bit word of sign bits per
//     replica (bit set <=> spin -1) straight from global memory and are expanded in
//     registers to bf16 +-1 (0x3F80 / 0xBF80), 8 spins per lane per MFMA.
// Matrix instruction: v_mfma_f32_32x32x16_bf16.  Operand layout (64 lanes):
//   A (32 x 16, rows = replicas): lane l holds row l%32, k = 8*(l/32) .. +7
//   B (16 x 32, cols = variables): lane l holds col l%32, k = 8*(l/32) .. +7
//   D (32 x 32): register v of lane l holds row 8*(v/4) + 4*(l/32) + v%4, col l%32.
// Epilogue: h = 2^e * acc + b, then the PA update on x, m (FP32, [Rp][np] row-major) and
// the new sign bits (one ballot per accumulator register -> two 32-bit words).
#include "qpa_internal.h"

namespace qpa {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = MF_BM, BN = MF_BN, BK = MF_BK;
constexpr int LDS_ROW = BK * 2 + 16;   // bytes per staged J row

__device__ __forceinline__ void pa_update(float h, float lam, float eta, float alpha, float &x,
                                          float &m) {
    float g = __fadd_rn(__fmul_rn(lam, x), h);
    float mn = __fsub_rn(__fmul_rn(alpha, m), __fmul_rn(eta, g));
    float y = __fadd_rn(x, mn);
    y = fminf(1.0f, fmaxf(-1.0f, y));
    m = mn;
    x = y;
}

// 8 sign bits (bit j <=> element j is -1) -> eight bf16 +-1 values.
__device__ __forceinline__ bf16x8 expand_spins(uint32_t byte) {
    u32x4 d;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t y = byte >> (2 * q);
        d[q] = 0x3F803F80u | ((y & 1u) << 15) | ((y & 2u) << 30);
    }
    return __builtin_bit_cast(bf16x8, d);
}

__global__ void __launch_bounds__(256) k_mfma_step(
    int64_t Rp, int64_t np, const uint16_t *__restrict__ Jb, const float *__restrict__ b,
    const CanonScalars *__restrict__ sc, const uint32_t *__restrict__ s_cur,
    uint32_t *__restrict__ s_nxt, float *__restrict__ x, float *__restrict__ m,
    float *__restrict__ h_last, int t, const float *__restrict__ lam, float eta, float alpha) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[2][BN * LDS_ROW];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t I0 = (int64_t)blockIdx.x * BN, R0 = (int64_t)blockIdx.y * BM;
    const int64_t wr0 = R0 + 32 * wv;
    const int64_t words = np / 32;
    const int nk = (int)(np / BK);

    // J stager: thread -> (row tid/2, 32 consecutive k at offset 32*(tid%2)) = 4 x 16 B
    const int lrow = tid >> 1, lhalf = tid & 1;
    const uint4 *gB = reinterpret_cast<const uint4 *>(Jb + (I0 + lrow) * np + lhalf * 32);
    const int lds_off = lrow * LDS_ROW + lhalf * 64;
    // spin bits of replica wr0 + lane%32: one 64-bit word per chunk
    const uint64_t *gA = reinterpret_cast<const uint64_t *>(s_cur + (wr0 + (lane & 31)) * words);

    f32x16 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[c][v] = 0.0f;

    uint4 breg[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) breg[e] = gB[e];
    uint64_t abits = gA[0];
#pragma unroll
    for (int e = 0; e < 4; ++e)
        *reinterpret_cast<uint4 *>(&lds[0][lds_off + 16 * e]) = breg[e];
    __syncthreads();

    const int half = lane >> 5;
    for (int kc = 0; kc < nk; ++kc) {
        uint64_t abits_next = 0;
        if (kc + 1 < nk) {
            const uint4 *src = gB + (int64_t)(kc + 1) * (BK / 8);
#pragma unroll
            for (int e = 0; e < 4; ++e) breg[e] = src[e];
            abits_next = gA[kc + 1];
        }
        const uint8_t *buf = lds[kc & 1];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t byte = (uint32_t)(abits >> (16 * q + 8 * half)) & 0xFFu;
            bf16x8 a = expand_spins(byte);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int row = 32 * c + (lane & 31);
                u32x4 bd = *reinterpret_cast<const u32x4 *>(buf + row * LDS_ROW + q * 32 +
                                                            half * 16);
                acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    a, __builtin_bit_cast(bf16x8, bd), acc[c], 0, 0, 0);
            }
        }
        if (kc + 1 < nk) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                *reinterpret_cast<uint4 *>(&lds[(kc + 1) & 1][lds_off + 16 * e]) = breg[e];
            abits = abits_next;
        }
        __syncthreads();
    }

    const float scale = sc->scale;
    const float lt = lam[t];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int64_t iv = I0 + 32 * c + (lane & 31);
        const float bi = b[iv];
        const int64_t wcol = (I0 + 32 * c) / 32;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int64_t r = wr0 + 8 * (v >> 2) + 4 * half + (v & 3);
            const int64_t g = r * np + iv;
            float h = __fadd_rn(__fmul_rn(acc[c][v], scale), bi);
            float xv = x[g], mv = m[g];
            pa_update(h, lt, eta, alpha, xv, mv);
            x[g] = xv;
            m[g] = mv;
            if (h_last) h_last[g] = h;
            uint64_t bal = __ballot(xv < 0.0f);
            uint32_t word = half ? (uint32_t)(bal >> 32) : (uint32_t)bal;
            if ((lane & 31) == 0) s_nxt[r * words + wcol] = word;
        }
    }
}

// sbits[r][w] bit j = (x[r][32w + j] < 0)
__global__ void __launch_bounds__(256) k_mfma_pack(int64_t Rp, int64_t np,
                                                   const float *__restrict__ x,
                                                   uint32_t *__restrict__ sbits) {
    const int64_t words = np / 32;
    const int64_t total = Rp * words;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = k / words, w = k - r * words;
        const float *xr = x + r * np + 32 * w;
        uint32_t bits = 0;
        for (int j = 0; j < 32; ++j) bits |= (xr[j] < 0.0f ? 1u : 0u) << j;
        sbits[k] = bits;
    }
}

}  // namespace

hipError_t launch_mfma_pack_spins(int64_t Rp, int64_t np, const float *x, uint32_t *sbits,
                                  hipStream_t st) {
    int64_t total = Rp * (np / 32);
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    k_mfma_pack<<<(unsigned)g, 256, 0, st>>>(Rp, np, x, sbits);
    return hipGetLastError();
}

hipError_t launch_mfma_step(int64_t Rp, int64_t np, const uint16_t *Jb, const float *b,
                            const CanonScalars *sc, const uint32_t *s_cur, uint32_t *s_nxt,
                            float *x, float *m, float *h_last, int32_t t, const float *lam,
                            float eta, float alpha, hipStream_t st) {
    if (Rp % BM || np % BN || np % BK) return hipErrorInvalidValue;
    dim3 grid((unsigned)(np / BN), (unsigned)(Rp / BM));
    k_mfma_step<<<grid, 256, 0, st>>>(Rp, np, Jb, b, sc, s_cur, s_nxt, x, m, h_last, t, lam, eta,
                                      alpha);
    return hipGetLastError();
}

}  // namespace qpa
