// Dense PA step on the CDNA4 matrix cores with BF16 couplings (App. B field J s + b,
// couplings stored as bf16(J / 2^e), FP32 accumulation, result scaled back by 2^e).
//
// One launch advances every replica by one step.  A workgroup owns an output tile of
// 128 replicas x 128 variables and has two kinds of waves:
//   * 4 matrix waves in a 2 x 2 arrangement: wave (wr, wc) accumulates replicas
//     64wr .. 64wr+63 against variables 64wc .. 64wc+63 (2 x 2 accumulators of 32 x 32)
//     over the whole reduction, walked in chunks of 128 variables;
//   * 4 state waves: they load the tile's x and m into registers when the launch starts,
//     so that this traffic overlaps the reduction, then wait for the field and run the
//     PA update and write x, m and the new sign bits.
// Chunks are staged through LDS with direct global->LDS loads issued by the matrix waves
// only (NST stages, NST-1 chunks in flight): per chunk the 128 x 128 bf16 block of J
// (8 loads of 16 bytes per lane and wave, each filling 4 rows of 256 bytes) and the
// 128 x 128 spin bits of the tile's replicas (2 loads of 4 bytes per lane and wave).
// Inside a J row the sixteen 16-byte pieces sit at position piece ^ (row % 16), so that
// the fragment reads of 16 consecutive rows fall on distinct banks.  One barrier per
// chunk publishes a stage and frees the one that is loaded next; the state waves take
// part in every barrier and issue no loads in between, so that the matrix waves' waits
// count their own loads only.  After the loop the raw sums go to the state waves
// through LDS (128 x 128 FP32, row-major).
//
// Spin bits ("chunk-major"): u32 word (kc * Rp + r) * 4 + q holds in bit j the sign of
// variable 128 kc + 32 q + j of replica r (bit set <=> spin -1), so that the spins of a
// tile's replicas for one chunk are one contiguous 2 KiB block.
//
// Matrix instruction: v_mfma_f32_32x32x16_bf16.  Operand layout (64 lanes):
//   A (32 x 16, rows = replicas): lane l holds row l%32, k = 8*(l/32) .. +7
//   B (16 x 32, cols = variables): lane l holds col l%32, k = 8*(l/32) .. +7
//   D (32 x 32): register v of lane l holds row 8*(v/4) + 4*(l/32) + v%4, col l%32.
#include "qpa_internal.h"

namespace qpa {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = MF_BM, BN = MF_BN;
constexpr int KC = 128;                      // reduction chunk (variables)
constexpr int JSTG = BN * KC * 2;            // J block of a stage: 128 rows x 256 bytes
constexpr int SSTG = BM * KC / 8;            // spin bits of a stage: 128 rows x 16 bytes
constexpr int STG = JSTG + SSTG;
constexpr int NST = 3;                       // stages
constexpr int LDS_BYTES = NST * STG;
constexpr int THREADS = 512;                 // 4 matrix waves + 4 state waves
constexpr int MW = 4;                        // matrix waves
static_assert(LDS_BYTES >= BM * BN * 4, "the field handoff reuses the stages");
static_assert(MF_NPAD % KC == 0, "np must be a multiple of the chunk");

__device__ __forceinline__ void pa_update(float h, float lam, float eta, float alpha, float &x,
                                          float &m) {
    float g = __fadd_rn(__fmul_rn(lam, x), h);
    float mn = __fsub_rn(__fmul_rn(alpha, m), __fmul_rn(eta, g));
    float y = __fadd_rn(x, mn);
    y = fminf(1.0f, fmaxf(-1.0f, y));
    m = mn;
    x = y;
}

typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));

// 8 sign bits (bit j <=> element j is -1) -> eight bf16 +-1 values:
// dword q holds elements 2q (low half) and 2q+1 (high half); a set bit sets the half's
// sign bit on top of 0x3F80 (= 1.0).  The byte is paired as 16-bit halves
// (byte, byte >> 1), so that one packed 16-bit shift by 15 - 2q brings bit 2q to the
// top of the low half and bit 2q+1 to the top of the high half; a mask keeps the two
// sign positions.  All full-rate ALU operations.
__device__ __forceinline__ bf16x8 expand_spins(uint32_t byte, uint32_t sign_mask) {
    // low half: byte (bit 15 also receives bit 0, which every shift below moves out);
    // high half: byte >> 1
    const uint32_t pair = (byte << 15) | byte;
    u32x4 d;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint16_t sh = (uint16_t)(15 - 2 * q);
        const u16x2 v = __builtin_bit_cast(u16x2, pair) << (u16x2){sh, sh};
        // (v & 0x80008000) | 0x3F803F80 in one instruction; the mask comes in a VGPR
        // because one VOP3 instruction can read only one scalar operand here
        uint32_t r;
        asm("v_and_or_b32 %0, %1, %2, %3"
            : "=v"(r)
            : "v"(__builtin_bit_cast(uint32_t, v)), "v"(sign_mask), "s"(0x3F803F80u));
        d[q] = r;
    }
    return __builtin_bit_cast(bf16x8, d);
}

typedef __attribute__((address_space(3))) void lds_void;

// Workgroup barrier without the memory fence of __syncthreads (which would also wait for
// every load in flight, including the chunks loaded ahead): the callers order their LDS
// traffic with the explicit waits below.
__device__ __forceinline__ void barrier() { asm volatile("s_barrier" ::: "memory"); }

// This wave's loads of all but the N youngest are done and its LDS accesses are complete,
// then the workgroup barrier.
template <int N> __device__ __forceinline__ void wait_barrier() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}

constexpr int LOADS_PER_CHUNK = 10;          // per matrix wave: 8 J pieces + 2 spin dwords

// One 128 x 128 output tile of one PA step: replicas R0 .. R0+127 (rows at or past
// `rlive` are padding: their state is neither read nor written and they report +1
// spins), variables I0 .. I0+127.  `lds` holds LDS_BYTES bytes.
__device__ __forceinline__ void mfma_tile_step(
    uint8_t *lds, int64_t np, int64_t Rp, int64_t I0, int64_t R0, int64_t rlive,
    const uint16_t *__restrict__ Jb, const float *__restrict__ b, float scale,
    const uint32_t *__restrict__ s_cur, uint32_t *__restrict__ s_nxt, float *__restrict__ x,
    float *__restrict__ m, float *__restrict__ h_last, float lt, float eta, float alpha) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nchunk = (int)(np / KC);
    float *hs = reinterpret_cast<float *>(lds);   // field sums of the tile, after the loop

    if (wave >= MW) {
        // ---- state waves: thread t owns column t % 128 of rows 2e + t / 128 ----
        const int t = tid - MW * 64;
        const int col = t & (BN - 1);
        const int rsub = __builtin_amdgcn_readfirstlane(t >> 7);
        const int64_t iv = I0 + col;
        const int64_t rmax = rlive - 1;
        float xv[BM / 2], mv[BM / 2];
#pragma unroll
        for (int e = 0; e < BM / 2; ++e) {
            // padding rows read a live row instead (never written back)
            const int64_t r = min(R0 + 2 * e + rsub, rmax);
            xv[e] = x[r * np + iv];
            mv[e] = m[r * np + iv];
        }
        const float bi = b[iv];
        for (int c = 0; c < nchunk; ++c) barrier();   // the matrix waves' chunks
        barrier();                                     // stages drained
        barrier();                                     // field sums in LDS
        // collect every load here, once, so that the stores below wait for nothing
#pragma unroll
        for (int e = 0; e < BM / 2; ++e) asm volatile("" ::"v"(xv[e]), "v"(mv[e]));
        asm volatile("" ::"v"(bi));
        const int64_t wbase = (I0 / KC) * Rp * 4 + 2 * ((wave - MW) & 1);
#pragma unroll
        for (int e = 0; e < BM / 2; ++e) {
            const int row = 2 * e + rsub;
            const int64_t r = R0 + row;
            const bool live = r < rlive;
            const float h = __fadd_rn(__fmul_rn(hs[row * BN + col], scale), bi);
            float xn = xv[e], mn = mv[e];
            pa_update(h, lt, eta, alpha, xn, mn);
            // this wave covers 64 consecutive variables of row r: one 64-bit spin word
            const uint64_t bal = __ballot(live && xn < 0.0f);
            if (live) {
                x[r * np + iv] = xn;
                m[r * np + iv] = mn;
                if (h_last) h_last[r * np + iv] = h;
            }
            if (lane == 0)
                *reinterpret_cast<uint64_t *>(s_nxt + wbase + r * 4) = bal;
        }
        return;
    }

    // ---- matrix waves ----
    const int wr = wave >> 1, wc = wave & 1;
    const int half = lane >> 5, l32 = lane & 31;
    // J: load u (0..7) of wave w fills LDS rows 32w + 4u + lane/16 at position lane % 16,
    // which holds piece (lane % 16) ^ (row % 16) of that row.
    const uint16_t *gJ[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int row = 32 * wave + 4 * u + (lane >> 4);
        gJ[u] = Jb + (I0 + row) * np + 8 * ((lane & 15) ^ (row & 15));
    }
    // spins: load e (0..1) of wave w fills bytes 512w + 256e + 4 lane of the 2 KiB block
    const uint32_t *gS = s_cur + R0 * 4 + 128 * wave + lane;
    const int64_t sstride = Rp * 4;                // u32 words between consecutive chunks
    auto stage = [&](int kc, int st) {
        kc = kc < nchunk ? kc : nchunk - 1;        // past the end: reload the last chunk
        uint8_t *dst = lds + st * STG;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            __builtin_amdgcn_global_load_lds(gJ[u] + (int64_t)kc * KC,
                                             (lds_void *)(dst + (8 * wave + u) * 1024), 16, 0, 0);
#pragma unroll
        for (int e = 0; e < 2; ++e)
            __builtin_amdgcn_global_load_lds(gS + (int64_t)kc * sstride + 64 * e,
                                             (lds_void *)(dst + JSTG + 512 * wave + 256 * e), 4,
                                             0, 0);
    };

    const uint32_t sign_mask = __builtin_amdgcn_readfirstlane(0x80008000u) + 0u * lane;
    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

#pragma unroll
    for (int s = 0; s < NST - 1; ++s) stage(s, s);
    for (int c = 0; c < nchunk; ++c) {
        // this wave's loads of chunk c have landed (the NST-2 younger chunks may not);
        // after the barrier every wave's have, and every wave is done with the stage of
        // chunk c-1, which is refilled next
        wait_barrier<(NST - 2) * LOADS_PER_CHUNK>();
        stage(c + NST - 1, (c + NST - 1) % NST);
        const uint8_t *src = lds + (c % NST) * STG;
        u32x4 sw[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            sw[i] = *reinterpret_cast<const u32x4 *>(src + JSTG + 16 * (64 * wr + 32 * i + l32));
#pragma unroll
        for (int q = 0; q < KC / 16; ++q) {
            u32x4 bq[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int row = 64 * wc + 32 * j + l32;
                const int pos = (2 * q + half) ^ (row & 15);
                bq[j] = *reinterpret_cast<const u32x4 *>(src + row * 256 + pos * 16);
            }
            bf16x8 a[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[i] = expand_spins((sw[i][q >> 1] >> (16 * (q & 1) + 8 * half)) & 0xFFu,
                                    sign_mask);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        a[i], __builtin_bit_cast(bf16x8, bq[j]), acc[i][j], 0, 0, 0);
        }
    }
    wait_barrier<0>();     // the trailing (redundant) loads have landed in every wave and
                           // every stage read is done: the stages can take the sums
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = 64 * wr + 32 * i + 8 * (v >> 2) + 4 * half + (v & 3);
                const int col = 64 * wc + 32 * j + l32;
                hs[row * BN + col] = acc[i][j][v];
            }
    wait_barrier<0>();     // field sums visible to the state waves
}

__global__ void __launch_bounds__(THREADS, 1) k_mfma_step(
    int64_t Rp, int64_t np, int64_t rlive, const uint16_t *__restrict__ Jb,
    const float *__restrict__ b, const CanonScalars *__restrict__ sc,
    const uint32_t *__restrict__ s_cur, uint32_t *__restrict__ s_nxt, float *__restrict__ x,
    float *__restrict__ m, float *__restrict__ h_last, int t, const float *__restrict__ lam,
    float eta, float alpha) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[LDS_BYTES];
    mfma_tile_step(lds, np, Rp, (int64_t)blockIdx.x * BN, (int64_t)blockIdx.y * BM, rlive, Jb,
                   b, sc->scale, s_cur, s_nxt, x, m, h_last, lam[t], eta, alpha);
}

// Many instances in one launch: block k runs tile k of the table.  Each tile points at
// its instance's couplings, bias, state and the two spin buffers (picked by step parity).
__global__ void __launch_bounds__(THREADS, 1) k_mfma_grouped(const MfmaTile *__restrict__ tiles,
                                                             int t, const float *__restrict__ lam,
                                                             float eta, float alpha) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[LDS_BYTES];
    const MfmaTile tl = tiles[blockIdx.x];
    const uint32_t *cur = (t & 1) ? tl.s1 : tl.s0;
    uint32_t *nxt = (t & 1) ? tl.s0 : tl.s1;
    mfma_tile_step(lds, tl.np, tl.Rp, tl.I0, tl.R0, tl.rlive, tl.Jb, tl.b, tl.sc->scale, cur, nxt,
                   tl.x, tl.m, nullptr, lam[t], eta, alpha);
}

// Chunk-major sign bits of x: word (kc * Rp + r) * 4 + q, bit j = (x[r][128kc + 32q + j] < 0)
__global__ void __launch_bounds__(256) k_mfma_pack(int64_t Rp, int64_t np,
                                                   const float *__restrict__ x,
                                                   uint32_t *__restrict__ sbits) {
    const int64_t words = np / 32;
    const int64_t total = Rp * words;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = k / words, wd = k - r * words;
        const float *xr = x + r * np + 32 * wd;
        uint32_t bits = 0;
        for (int j = 0; j < 32; ++j) bits |= (xr[j] < 0.0f ? 1u : 0u) << j;
        sbits[((wd >> 2) * Rp + r) * 4 + (wd & 3)] = bits;
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
    if (Rp % BM || np % MF_NPAD || np <= 0 || rlive < 1 || rlive > Rp)
        return hipErrorInvalidValue;
    dim3 grid((unsigned)(np / BN), (unsigned)(Rp / BM));
    k_mfma_step<<<grid, THREADS, 0, st>>>(Rp, np, rlive, Jb, b, sc, s_cur, s_nxt, x, m, h_last,
                                          t, lam, eta, alpha);
    return hipGetLastError();
}

hipError_t launch_mfma_grouped(const MfmaTile *tiles, int32_t ntiles, int32_t t,
                               const float *lam, float eta, float alpha, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    k_mfma_grouped<<<(unsigned)ntiles, THREADS, 0, st>>>(tiles, t, lam, eta, alpha);
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
