// Dense PA step on the CDNA4 matrix cores with BF16 couplings (App. B field J s + b,
// couplings stored as bf16(J / 2^e), FP32 accumulation, result scaled back by 2^e).
//
// One launch advances every replica by one step.  A workgroup owns an output tile of
// 128 replicas x 128 variables and splits the reduction dimension over its 4 waves:
// wave w accumulates the whole tile (4 x 4 accumulators of 32x32 in AGPRs) over
// k in [w*np/4, (w+1)*np/4), walking it in chunks of 64.
//   * each wave stages its own chunk -- the 128 x 64 bf16 block of J and the 128 spin
//     words (sign bits, bit set <=> spin -1, one 64-bit word per 64 variables and replica
//     row) -- into a wave-private LDS stage (two stages) with direct global->LDS loads:
//     16 loads of 16 bytes per lane for J, each covering 8 full 128-byte rows, and 4 of
//     4 bytes for the spin words.  Every operand of the tile is fetched once per
//     workgroup, coalesced, without passing through registers; the only wait is one
//     vmcnt(0) per chunk, a whole chunk of MFMAs after the loads were issued.  Inside
//     a J row the eight 16-byte pieces sit at position (piece ^ (row % 8)), so that the
//     fragment reads of 8 consecutive lanes (8 consecutive rows) hit distinct banks.
//   * all 16 B fragments and 4 spin words of a chunk are read from LDS before the next
//     chunk's loads are issued; the 8 bits of a fragment row are expanded to bf16 +-1
//     (0x3F80 / 0xBF80) and reused by the 4 MFMAs of that row.
// After the loop the four partial tiles are summed through LDS so that wave w holds
// replicas 32w .. 32w+31 of the tile for all 128 variables, then runs the PA update.
//
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

constexpr int BM = MF_BM, BN = MF_BN;
constexpr int JST = BN * 128;                // J bytes of a wave stage: 128 rows x 64 bf16
constexpr int STG = JST + BM * 8;            // + one 64-bit spin word per replica row

__device__ __forceinline__ void pa_update(float h, float lam, float eta, float alpha, float &x,
                                          float &m) {
    float g = __fadd_rn(__fmul_rn(lam, x), h);
    float mn = __fsub_rn(__fmul_rn(alpha, m), __fmul_rn(eta, g));
    float y = __fadd_rn(x, mn);
    y = fminf(1.0f, fmaxf(-1.0f, y));
    m = mn;
    x = y;
}

// 8 sign bits (bit j <=> element j is -1) -> eight bf16 +-1 values:
// dword q holds elements 2q (low half) and 2q+1 (high half); a set bit sets the half's
// sign bit on top of 0x3F80 (= 1.0).
__device__ __forceinline__ bf16x8 expand_spins(uint32_t byte) {
    u32x4 d;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t y = byte >> (2 * q);
        uint32_t spread = (y << 15) | (y << 30);
        d[q] = (spread & 0x80008000u) | 0x3F803F80u;
    }
    return __builtin_bit_cast(bf16x8, d);
}

typedef __attribute__((address_space(3))) void lds_void;

// One 128 x 128 output tile of one PA step: replicas R0 .. R0+127 (rows at or past
// `rlive` are padding: no state traffic), variables I0 .. I0+127.  `lds` holds
// 4 * 2 * STG bytes.
__device__ __forceinline__ void mfma_tile_step(
    uint8_t *lds, int64_t np, int64_t I0, int64_t R0, int64_t rlive,
    const uint16_t *__restrict__ Jb, const float *__restrict__ b, float scale,
    const uint64_t *__restrict__ s_cur, uint32_t *__restrict__ s_nxt, float *__restrict__ x,
    float *__restrict__ m, float *__restrict__ h_last, float lt, float eta, float alpha) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int half = lane >> 5, l32 = lane & 31;
    const int64_t kq = np / 4;                 // reduction length of one wave
    const int64_t kb = (int64_t)w * kq;
    const int nchunk = (int)(kq / 64);
    const int64_t wpr = np / 64;               // spin words per replica row
    uint8_t *mine = lds + w * 2 * STG;

    // J: load e (0..15) fills rows 8e .. 8e+7 of a stage; lane l covers row 8e + l/8 and
    // stores at position l%8 the piece (l%8) ^ (row%8) = (l%8) ^ (l/8).
    const uint16_t *gJ = Jb + (I0 + (lane >> 3)) * np + kb + 8 * ((lane & 7) ^ (lane >> 3));
    // spin words: load e (0..3) fills rows 32e .. 32e+31; lane l covers row 32e + l/2,
    // 32-bit half l%2 of that row's 64-bit word, so a row's word is contiguous in LDS.
    const uint32_t *gS = reinterpret_cast<const uint32_t *>(s_cur + (R0 + (lane >> 1)) * wpr +
                                                            kb / 64) + (lane & 1);
    auto stage = [&](int kc, int st) {
        kc = kc < nchunk ? kc : nchunk - 1;   // past the end: reload the last chunk
        const uint16_t *srcJ = gJ + (int64_t)kc * 64;
        const uint32_t *srcS = gS + 2 * (int64_t)kc;
        uint8_t *dst = mine + st * STG;
#pragma unroll
        for (int e = 0; e < 16; ++e)
            __builtin_amdgcn_global_load_lds(srcJ + (int64_t)8 * e * np,
                                             (lds_void *)(dst + e * 1024), 16, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e)
            __builtin_amdgcn_global_load_lds(srcS + (int64_t)32 * e * 2 * wpr,
                                             (lds_void *)(dst + JST + e * 256), 4, 0, 0);
    };

    f32x16 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

    stage(0, 0);
    for (int c = 0; c < nchunk; ++c) {
        // chunk c was requested one chunk ago: wait for it here, and keep every LDS read
        // of the chunk below this point
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        const uint8_t *src = mine + (c & 1) * STG;
        u32x4 bf[4][4];                         // [k step q][variable fragment j]
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = 32 * j + l32;
                const int pos = (2 * q + half) ^ (row & 7);
                bf[q][j] = *reinterpret_cast<const u32x4 *>(src + row * 128 + (pos << 4));
            }
        uint64_t aw[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            aw[i] = *reinterpret_cast<const uint64_t *>(src + JST + 8 * (32 * i + l32));
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        stage(c + 1, (c + 1) & 1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            bf16x8 a[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                a[i] = expand_spins((uint32_t)(aw[i] >> (16 * q + 8 * half)) & 0xFFu);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        a[i], __builtin_bit_cast(bf16x8, bf[q][j]), acc[i][j], 0, 0, 0);
        }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // the last (redundant) loads landed
    __syncthreads();

    // sum the partial tiles: wave w ends up with replica fragment w (all 4 variable
    // fragments), adding the other waves' partials in ascending wave order.
    float *red = reinterpret_cast<float *>(lds);
    f32x16 fin[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (i != w)
#pragma unroll
                for (int v = 0; v < 16; ++v) red[((i * 4 + w) * 16 + v) * 64 + lane] = acc[i][j][v];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (i == w) fin[j] = acc[i][j];
#pragma unroll
        for (int src = 0; src < 4; ++src)
            if (src != w)
#pragma unroll
                for (int v = 0; v < 16; ++v) fin[j][v] += red[((w * 4 + src) * 16 + v) * 64 + lane];
        __syncthreads();
    }

    const int64_t wrow = np / 32;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t iv = I0 + 32 * j + l32;
        const float bi = b[iv];
        const int64_t wcol = (I0 + 32 * j) / 32;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int64_t r = R0 + 32 * w + 8 * (v >> 2) + 4 * half + (v & 3);
            const int64_t g = r * np + iv;
            float xv = 0.0f;
            if (r < rlive) {
                float h = __fadd_rn(__fmul_rn(fin[j][v], scale), bi);
                float mv = m[g];
                xv = x[g];
                pa_update(h, lt, eta, alpha, xv, mv);
                x[g] = xv;
                m[g] = mv;
                if (h_last) h_last[g] = h;
            }
            uint64_t bal = __ballot(xv < 0.0f);
            uint32_t word = half ? (uint32_t)(bal >> 32) : (uint32_t)bal;
            if (l32 == 0) s_nxt[r * wrow + wcol] = word;
        }
    }
}

__global__ void __launch_bounds__(256, 1) k_mfma_step(
    int64_t Rp, int64_t np, int64_t rlive, const uint16_t *__restrict__ Jb,
    const float *__restrict__ b, const CanonScalars *__restrict__ sc,
    const uint64_t *__restrict__ s_cur, uint32_t *__restrict__ s_nxt, float *__restrict__ x,
    float *__restrict__ m, float *__restrict__ h_last, int t, const float *__restrict__ lam,
    float eta, float alpha) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[4 * 2 * STG];
    mfma_tile_step(lds, np, (int64_t)blockIdx.x * BN, (int64_t)blockIdx.y * BM, rlive, Jb, b,
                   sc->scale, s_cur, s_nxt, x, m, h_last, lam[t], eta, alpha);
}

// Many instances in one launch: block k runs tile k of the table.  Each tile points at
// its instance's couplings, bias, state and the two spin buffers (picked by step parity).
__global__ void __launch_bounds__(256, 1) k_mfma_grouped(const MfmaTile *__restrict__ tiles,
                                                         int t, const float *__restrict__ lam,
                                                         float eta, float alpha) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[4 * 2 * STG];
    const MfmaTile tl = tiles[blockIdx.x];
    const uint64_t *cur = reinterpret_cast<const uint64_t *>((t & 1) ? tl.s1 : tl.s0);
    uint32_t *nxt = (t & 1) ? tl.s0 : tl.s1;
    mfma_tile_step(lds, tl.np, tl.I0, tl.R0, tl.rlive, tl.Jb, tl.b, tl.sc->scale, cur, nxt, tl.x,
                   tl.m, nullptr, lam[t], eta, alpha);
}

// sbits[r][w] bit j = (x[r][32w + j] < 0)
__global__ void __launch_bounds__(256) k_mfma_pack(int64_t Rp, int64_t np,
                                                   const float *__restrict__ x,
                                                   uint32_t *__restrict__ sbits) {
    const int64_t words = np / 32;
    const int64_t total = Rp * words;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = k / words, wd = k - r * words;
        const float *xr = x + r * np + 32 * wd;
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

hipError_t launch_mfma_step(int64_t Rp, int64_t np, int64_t rlive, const uint16_t *Jb,
                            const float *b, const CanonScalars *sc, const uint32_t *s_cur,
                            uint32_t *s_nxt, float *x, float *m, float *h_last, int32_t t,
                            const float *lam, float eta, float alpha, hipStream_t st) {
    if (Rp % BM || np % MF_NPAD) return hipErrorInvalidValue;
    dim3 grid((unsigned)(np / BN), (unsigned)(Rp / BM));
    k_mfma_step<<<grid, 256, 0, st>>>(Rp, np, rlive, Jb, b, sc,
                                      reinterpret_cast<const uint64_t *>(s_cur), s_nxt, x, m,
                                      h_last, t, lam, eta, alpha);
    return hipGetLastError();
}

hipError_t launch_mfma_grouped(const MfmaTile *tiles, int32_t ntiles, int32_t t,
                               const float *lam, float eta, float alpha, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    k_mfma_grouped<<<(unsigned)ntiles, 256, 0, st>>>(tiles, t, lam, eta, alpha);
    return hipGetLastError();
}

// Dense BF16 copy of a CSR instance: Jb[i][j] = bf16(w_ij * 2^-e) for the stored
// off-diagonal entries (zero elsewhere; the caller clears Jb first).
template <typename TW, typename TI>
__global__ void __launch_bounds__(256) k_csr_to_bf16(int64_t n, int64_t np,
                                                     const int32_t *__restrict__ rp,
                                                     const TI *__restrict__ col,
                                                     const TW *__restrict__ w,
                                                     const CanonScalars *__restrict__ sc,
                                                     uint16_t *__restrict__ Jb) {
    const float inv = sc->inv_scale;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int64_t j = (int64_t)col[k];
            if (j == i) continue;
            uint32_t u = __float_as_uint(__fmul_rn((float)w[k], inv));
            u += 0x7fffu + ((u >> 16) & 1u);
            Jb[i * np + j] = (uint16_t)(u >> 16);
        }
    }
}

hipError_t launch_csr_to_bf16(const qpa_problem &p, int64_t np, const CanonScalars *sc,
                              uint16_t *Jb, hipStream_t st) {
    hipError_t e = hipMemsetAsync(Jb, 0, sizeof(uint16_t) * (size_t)(np * np), st);
    if (e != hipSuccess) return e;
    int64_t g = (p.n + 255) / 256;
    auto run = [&](auto wtag, auto itag) {
        using TW = decltype(wtag);
        using TI = decltype(itag);
        k_csr_to_bf16<TW, TI><<<(unsigned)g, 256, 0, st>>>(
            p.n, np, p.row_ptr, static_cast<const TI *>(p.col),
            static_cast<const TW *>(p.weights), sc, Jb);
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

}  // namespace qpa
