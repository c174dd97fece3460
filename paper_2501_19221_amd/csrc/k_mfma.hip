// Dense PA step on the CDNA4 matrix cores with BF16 couplings (App. B field J s + b,
// couplings stored as bf16(J / 2^e), FP32 accumulation, result scaled back by 2^e).
//
// One launch advances every replica by one step.  A workgroup owns an output tile of
// 128 replicas x 128 variables and has 16 waves, four per SIMD:
//   * 8 matrix waves: a 2 x 2 arrangement of 64 x 64 sub-tiles, each worked on by two
//     waves that split every chunk's eight k steps between them (steps 0..3 and 4..7),
//     so that every SIMD runs two matrix waves whose instruction streams interleave (one
//     wave alone cannot issue its operand expansion while its matrix ops run); each wave
//     keeps 2 x 2 accumulators of 32 x 32 and the two halves are summed in LDS at the end;
//   * 8 state waves: they load the tile's x and m into registers while the reduction
//     runs, then wait for the field and run the PA update and write x, m and the spins.
// Chunks are staged through LDS with direct global->LDS loads issued by the matrix waves
// only (NST stages, NST-1 chunks in flight): per chunk the 128 x 128 bf16 block of J
// (4 loads of 16 bytes per lane and wave, each filling 4 rows of 256 bytes) and the spins
// of the tile's 128 replicas for those 128 variables (1 load of 16 bytes per lane and
// wave, 64 bytes per replica).
// Inside a J row the sixteen 16-byte pieces sit at position piece ^ (row % 16), and inside
// a replica's 64 spin bytes the four 16-byte pieces at (piece + row / 4) % 4, so that the
// fragment reads of 16 consecutive rows fall on distinct banks.  One barrier per
// chunk publishes a stage and frees the one that is loaded next; the state waves take
// part in every barrier and issue no loads in between, so that the matrix waves' waits
// count their own loads only.  After the loop the raw sums go to the state waves
// through LDS, one 128 x 128 FP32 buffer per k half (rows padded to 136 so that the two
// halves of a wave's stores use different banks), added by the state waves.
//
// Spins ("pair words", chunk-major): for replica r and chunk kc (variables 128 kc ..
// 128 kc + 127) there are 16 u32 words at (kc * Rp + r) * 16.  Word 8 h + q covers the
// eight variables 128 kc + 16 q + 8 h + j (j = 0..7) -- exactly the k values of one lane
// half h of the matrix instruction's operand at k step q -- as the byte B (bit j set <=>
// spin -1) in its low half and B >> 1 in its high half, the form the sign expansion
// starts from.  The state waves write this form once per step; each word is expanded by
// every tile of its replicas' row, so work moved into the writer is saved many times.
//
// Matrix instruction: v_mfma_f32_32x32x16_bf16.  Operand layout (64 lanes):
//   A (32 x 16, rows = replicas): lane l holds row l%32, k = 8*(l/32) .. +7
//   B (16 x 32, cols = variables): lane l holds col l%32, k = 8*(l/32) .. +7
//   D (32 x 32): register v of lane l holds row 8*(v/4) + 4*(l/32) + v%4, col l%32.
#include "qpa_internal.h"

#include <algorithm>

namespace qpa {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = MF_BM, BN = MF_BN;
constexpr int KC = 128;                      // reduction chunk (variables)
constexpr int JSTG = BN * KC * 2;            // J block of a stage: 128 rows x 256 bytes
constexpr int SSTG = BM * 64;                // spin words of a stage: 128 rows x 64 bytes
constexpr int STG = JSTG + SSTG;
constexpr int NST = 4;                       // stages
constexpr int LDS_BYTES = NST * STG;
// Integer couplings with |J| <= 127 (exact in int8) run on tiles of 64 replicas x 256
// variables (see the int8 section below): J rows of 128 bytes per chunk, spins one byte per
// (replica, variable) (+1 = 0x01, -1 = 0xFF), chunk-major (128 bytes per replica and
// chunk), v_mfma_i32_32x32x32_i8 with exact int32 sums.
constexpr int BM8 = MF_BM8, BN8 = MF_BN8;    // 64 replicas x 256 variables
constexpr int JSTG8 = BN8 * KC;              // 256 rows x 128 bytes
constexpr int SSTG8 = BM8 * KC;              // 64 replicas x 128 bytes
constexpr int STG8 = JSTG8 + SSTG8;
constexpr int NST8 = 4;
constexpr int HS8 = BN8 + 8;                 // row stride of the int8 handoff (int32)
constexpr int SR8 = BM8 / 2;                 // rows per state thread of an int8 tile
static_assert(NST8 * STG8 <= LDS_BYTES, "int8 stages fit the same LDS");
static_assert(2 * BM8 * HS8 * 4 <= LDS_BYTES, "the int8 handoff's two partial-sum buffers");
static_assert(BN8 % KC == 0 && BN8 / 16 == 16, "16 row groups of 16 per int8 tile");
constexpr int HS = BN + 8;                   // row stride of the field handoff (floats)
constexpr int THREADS = 1024;                // 8 matrix waves + 8 state waves
constexpr int MW = 8;                        // matrix waves
constexpr int SR = BM / 4;                   // rows per state thread
static_assert(LDS_BYTES >= BM * HS * 4, "the field handoff reuses the stages");
static_assert(LDS_BYTES >= 2 * BM * HS * 4, "the two k halves' handoff buffers");
static_assert(LDS_BYTES <= 160 * 1024, "LDS of one workgroup");
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

// Pair word (low half: byte B of 8 sign bits, bit j <=> element j is -1; high half:
// B >> 1) -> eight bf16 +-1 values: dword q holds elements 2q (low half) and 2q+1 (high
// half); a set bit sets the half's sign bit on top of 0x3F80 (= 1.0).  One packed 16-bit
// shift by 15 - 2q brings bit 2q to the top of the low half and bit 2q+1 to the top of
// the high half; a mask keeps the two sign positions.  Two full-rate operations per dword.
__device__ __forceinline__ uint32_t spin_pair(uint32_t byte) { return byte | ((byte >> 1) << 16); }

__device__ __forceinline__ bf16x8 expand_spins(uint32_t pair, uint32_t sign_mask) {
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

constexpr int LOADS_PER_CHUNK = 5;           // per matrix wave: 4 J pieces + 1 spin piece

// The tile of a workgroup: replicas R0 .. R0+127 (rows at or past `rlive` are padding:
// their state is neither read nor written and they report +1 spins), variables
// I0 .. I0+127 of an instance with np padded variables and Rp padded replicas.
struct Tile {
    int64_t np, Rp, I0, R0, rlive;
    const uint16_t *Jb;
    const float *b;
    float scale;
    float *x, *m;
    const uint32_t *E = nullptr;     // sparse int8 tiles: entries and block offsets
    const int32_t *O = nullptr;
};

// ---- matrix waves: the reduction of one step, left in LDS as raw sums --------------
// Executes nchunk + 2 workgroup barriers (the state waves execute as many).
__device__ __forceinline__ void matrix_step(uint8_t *lds, const Tile &tl, int nchunk,
                                            const uint32_t *__restrict__ s_cur, int wave,
                                            int lane) {
    const int64_t np = tl.np, I0 = tl.I0, R0 = tl.R0;
    const uint16_t *__restrict__ Jb = tl.Jb;
    float *hs = reinterpret_cast<float *>(lds);
    const int kh = wave >> 2;                      // k steps 4 kh .. 4 kh + 3 of a chunk
    const int wr = (wave >> 1) & 1, wc = wave & 1;
    const int half = lane >> 5, l32 = lane & 31;
    // J: load u (0..3) of wave w fills LDS rows 16w + 4u + lane/16 at position lane % 16,
    // which holds piece (lane % 16) ^ (row % 16) of that row.  Addresses are a
    // wave-uniform base plus 32-bit lane offsets (fewer registers than 64-bit pointers).
    const uint16_t *Jw = Jb + (I0 + 16 * wave) * np;
    uint32_t oJ[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int r = 4 * u + (lane >> 4);         // row - 16 w, and row % 16 == r % 16
        oJ[u] = (uint32_t)r * (uint32_t)np + 8u * (uint32_t)((lane & 15) ^ (r & 15));
    }
    // spins: the load of wave w fills bytes 1024w + 16 lane of the 8 KiB block of the
    // tile's replicas (64 bytes per replica, in replica order): row 16w + lane/4,
    // position lane % 4, which holds piece (lane - row / 4) % 4
    const uint32_t *Sw = s_cur + (R0 + 16 * wave) * 16;
    const uint32_t oS = (uint32_t)(lane >> 2) * 16u +
                        4u * (uint32_t)(((lane & 3) - ((lane >> 4) & 3)) & 3);
    const int64_t sstride = tl.Rp * 16;            // u32 words between consecutive chunks
    auto stage = [&](int kc, int st) {
        kc = kc < nchunk ? kc : nchunk - 1;        // past the end: reload the last chunk
        uint8_t *dst = lds + st * STG;
        const uint16_t *jc = Jw + (int64_t)kc * KC;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            __builtin_amdgcn_global_load_lds(jc + oJ[u],
                                             (lds_void *)(dst + (4 * wave + u) * 1024), 16, 0, 0);
        __builtin_amdgcn_global_load_lds(Sw + (int64_t)kc * sstride + oS,
                                         (lds_void *)(dst + JSTG + 1024 * wave), 16, 0, 0);
    };

    const uint32_t sign_mask = __builtin_amdgcn_readfirstlane(0x80008000u) + 0u * lane;
    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

    // the products of chunk c from its stage
    auto multiply = [&](int c) {
        const uint8_t *src = lds + (c % NST) * STG;
        // this lane's 4 pair words (k steps 4 kh .. 4 kh + 3 of its half) per replica
        // fragment: piece 2 half + kh of the replica's 64 bytes
        u32x4 sw[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int row = 64 * wr + 32 * i + l32;
            const int pos = (2 * half + kh + (row >> 2)) & 3;
            sw[i] = *reinterpret_cast<const u32x4 *>(src + JSTG + 64 * row + 16 * pos);
        }
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int q = 4 * kh + qq;
            u32x4 bq[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int row = 64 * wc + 32 * j + l32;
                const int pos = (2 * q + half) ^ (row & 15);
                bq[j] = *reinterpret_cast<const u32x4 *>(src + row * 256 + pos * 16);
            }
            bf16x8 a[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = expand_spins(sw[i][qq], sign_mask);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        a[i], __builtin_bit_cast(bf16x8, bq[j]), acc[i][j], 0, 0, 0);
        }
    };
#pragma unroll
    for (int s = 0; s < NST - 1; ++s) stage(s, s);
    for (int c = 0; c < nchunk; ++c) {
        // this wave's loads of chunk c have landed (the NST-2 younger chunks may not);
        // after the barrier every wave's have, and every wave is done with the stage of
        // chunk c-1, which is refilled next
        wait_barrier<(NST - 2) * LOADS_PER_CHUNK>();
        stage(c + NST - 1, (c + NST - 1) % NST);
        multiply(c);
    }
    wait_barrier<0>();     // the trailing (redundant) loads have landed in every wave and
                           // every stage read is done: the stages can take the sums
    // each k half stores its sums into its own buffer (the state waves add the two, first
    // half + second half), in one pass
    float *hp0 = hs + kh * (BM * HS);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = 64 * wr + 32 * i + 8 * (v >> 2) + 4 * half + (v & 3);
                const int col = 64 * wc + 32 * j + l32;
                hp0[row * HS + col] = acc[i][j][v];
            }
    wait_barrier<0>();      // partial sums stored
}

// ---- state waves: thread t (0..511) owns column t % 128 of rows 4e + t / 128 ---------
// Row pointers are wave-uniform and advanced one row pair at a time through an opaque
// step, so that the compiler computes each address when it is used instead of holding
// all 64 in scalar registers.
template <typename P> __device__ __forceinline__ P *next_rows(P *p, int64_t stride) {
    P *q = p + stride;
    asm volatile("" : "+s"(q));
    return q;
}

struct StateRegs {
    float xv[SR], mv[SR];
    float bi;
};

// Loads the tile's x, m and b, spread over the matrix waves' nchunk chunk barriers (a
// few elements before each), so that this traffic shares the memory system with the
// chunk loads instead of delaying the first chunks.  Rows past rlive are padding: they
// are not read and take zeros.  Row pointers are wave-uniform, so that each load is a
// scalar base plus the lane's column.  Executes nchunk barriers.  NTL: non-temporal loads
// (the grouped batch step).
template <bool NTL>
__device__ __forceinline__ void state_load(StateRegs &st, const Tile &tl, int nchunk, int t) {
    const int col = t & (BN - 1);
    const int rsub = __builtin_amdgcn_readfirstlane(t >> 7);
    const int per = (SR + nchunk - 1) / nchunk;
    const float *xr = tl.x + (tl.R0 + rsub) * tl.np + tl.I0;
    const float *mr = tl.m + (tl.R0 + rsub) * tl.np + tl.I0;
    int passed = 0;
#pragma unroll
    for (int e = 0; e < SR; ++e) {
        if (e > 0 && e % per == 0 && passed < nchunk) {
            barrier();
            ++passed;
        }
        // padding rows (uniform per wave) are not read: they start from zero each step
        const bool live = tl.R0 + 4 * e + rsub < tl.rlive;
        st.xv[e] = live ? (NTL ? __builtin_nontemporal_load(&xr[col]) : xr[col]) : 0.0f;
        st.mv[e] = live ? (NTL ? __builtin_nontemporal_load(&mr[col]) : mr[col]) : 0.0f;
        xr = next_rows(xr, 4 * tl.np);
        mr = next_rows(mr, 4 * tl.np);
    }
    st.bi = tl.b[tl.I0 + col];
    for (; passed < nchunk; ++passed) barrier();   // the remaining chunks
}

// Waits for the loads of state_load, once, so that later stores wait for nothing.
__device__ __forceinline__ void state_collect(StateRegs &st) {
#pragma unroll
    for (int e = 0; e < SR; ++e) asm volatile("" ::"v"(st.xv[e]), "v"(st.mv[e]));
    asm volatile("" ::"v"(st.bi));
}

// The PA update of the tile from the field sums in LDS, then the new spins as pair words.
// Rows are taken in groups of 8 with no branch inside the loop (the field reads of a group
// are issued together); lane 2g + ln keeps the ballot of row g of each group, and after
// the loop lanes 0..15 turn them into 16-byte stores (the even (ln = 0) or odd (ln = 1)
// bytes of their row).  With h_last the fields are stored by a second pass.  Executes no
// barrier.
__device__ __forceinline__ void state_update(StateRegs &st, const Tile &tl, const float *hs,
                                             uint32_t *__restrict__ s_nxt,
                                             float *__restrict__ h_last, int t, int wave,
                                             int lane, float lt, float eta, float alpha) {
    const int col = t & (BN - 1);
    const int rsub = __builtin_amdgcn_readfirstlane(t >> 7);
    {
    const int u_mine = (lane >> 1) & 7;
    uint64_t mine[SR / 8];
#pragma unroll
    for (int g = 0; g < SR / 8; ++g) {
        float hv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = (4 * (8 * g + u) + rsub) * HS + col;
            hv[u] = hs[k] + hs[BM * HS + k];          // first k half + second k half
        }
        uint64_t bal[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = 8 * g + u;
            const bool live = tl.R0 + 4 * e + rsub < tl.rlive;      // uniform per wave
            const float h = __fadd_rn(__fmul_rn(hv[u], tl.scale), st.bi);
            pa_update(h, lt, eta, alpha, st.xv[e], st.mv[e]);
            bal[u] = __ballot(live && st.xv[e] < 0.0f);
        }
        mine[g] = bal[0];
#pragma unroll
        for (int k = 1; k < 8; ++k) mine[g] = u_mine == k ? bal[k] : mine[g];
    }
    // this wave covers variables 64 c2 .. 64 c2 + 63 of the chunk: ballot byte k of a row
    // is word 8 (k & 1) + 4 c2 + k / 2 of the replica's 16 pair words
    if (lane < 16) {
        const int c2 = (wave - MW) & 1;
        const int ln = lane & 1;
        uint32_t *wrow = s_nxt + ((tl.I0 / KC) * tl.Rp + tl.R0 + rsub) * 16 + 4 * c2 + 8 * ln;
#pragma unroll
        for (int g = 0; g < SR / 8; ++g) {
            u32x4 wq;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                wq[k] = spin_pair((uint32_t)(mine[g] >> (8 * (2 * k + ln))) & 0xFFu);
            *reinterpret_cast<u32x4 *>(wrow + 64 * (8 * g + u_mine)) = wq;
        }
    }
    }
    if (h_last) {
        float *hr = h_last + (tl.R0 + rsub) * tl.np + tl.I0;
#pragma unroll
        for (int e = 0; e < SR; ++e) {
            if (tl.R0 + 4 * e + rsub < tl.rlive)
                hr[col] = __fadd_rn(__fmul_rn(hs[(4 * e + rsub) * HS + col] +
                                                  hs[BM * HS + (4 * e + rsub) * HS + col],
                                              tl.scale),
                                    st.bi);
            hr = next_rows(hr, 4 * tl.np);
        }
    }
}

// NT: non-temporal stores.  Measured: 1.6 % faster for the single-instance step; for the
// grouped batch step (a batch's state, couplings and spins are more than the caches hold
// between steps) non-temporal stores and loads (NTL in state_load) together 6 % faster.
template <bool NT>
__device__ __forceinline__ void state_store(const StateRegs &st, const Tile &tl, int t) {
    const int col = t & (BN - 1);
    const int rsub = __builtin_amdgcn_readfirstlane(t >> 7);
    float *xr = tl.x + (tl.R0 + rsub) * tl.np + tl.I0;
    float *mr = tl.m + (tl.R0 + rsub) * tl.np + tl.I0;
#pragma unroll
    for (int e = 0; e < SR; ++e) {
        if (tl.R0 + 4 * e + rsub < tl.rlive) {
            if (NT) {
                __builtin_nontemporal_store(st.xv[e], &xr[col]);
                __builtin_nontemporal_store(st.mv[e], &mr[col]);
            } else {
                xr[col] = st.xv[e];
                mr[col] = st.mv[e];
            }
        }
        xr = next_rows(xr, 4 * tl.np);
        mr = next_rows(mr, 4 * tl.np);
    }
}

// One PA step of one BF16 tile: matrix and state waves side by side.
template <bool NT, bool NTL = false>
__device__ __forceinline__ void mfma_tile_step(uint8_t *lds, const Tile &tl,
                                               const uint32_t *__restrict__ s_cur,
                                               uint32_t *__restrict__ s_nxt,
                                               float *__restrict__ h_last, float lt, float eta,
                                               float alpha) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nchunk = (int)(tl.np / KC);
    if (wave >= MW) {
        const int t = tid - MW * 64;
        StateRegs st;
        state_load<NTL>(st, tl, nchunk, t);
        barrier();                                     // stages drained
        barrier();                                     // partial sums stored
        state_collect(st);
        state_update(st, tl, reinterpret_cast<const float *>(lds), s_nxt, h_last, t, wave, lane,
                     lt, eta, alpha);
        state_store<NT>(st, tl, t);
        return;
    }
    matrix_step(lds, tl, nchunk, s_cur, wave, lane);
}

__global__ void __launch_bounds__(THREADS, 1) k_mfma_step(
    int64_t Rp, int64_t np, int64_t rlive, const uint16_t *__restrict__ Jb,
    const float *__restrict__ b, const CanonScalars *__restrict__ sc,
    const uint32_t *__restrict__ s_cur, uint32_t *__restrict__ s_nxt, float *__restrict__ x,
    float *__restrict__ m, float *__restrict__ h_last, int t, const float *__restrict__ lam,
    float eta, float alpha) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[LDS_BYTES];
    const Tile tl{np, Rp, (int64_t)blockIdx.x * BN, (int64_t)blockIdx.y * BM, rlive, Jb, b,
                  sc->scale, x, m};
    mfma_tile_step<true>(lds, tl, s_cur, s_nxt, h_last, lam[t], eta, alpha);
}

// Many instances in one launch: block k runs tile k of the table.  Each tile points at
// its instance's couplings, bias, state and the two spin buffers (picked by step parity).
__global__ void __launch_bounds__(THREADS, 1) k_mfma_grouped(const MfmaTile *__restrict__ tiles,
                                                             int t, const float *__restrict__ lam,
                                                             float eta, float alpha) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[LDS_BYTES];
    const MfmaTile mt = tiles[blockIdx.x];
    if (mt.np == 0) return;      // filler entry of the compute-die-ordered table
    const uint32_t *cur = (t & 1) ? mt.s1 : mt.s0;
    uint32_t *nxt = (t & 1) ? mt.s0 : mt.s1;
    const Tile tl{mt.np, mt.Rp, mt.I0, mt.R0, mt.rlive, mt.Jb, mt.b, mt.sc->scale, mt.x, mt.m};
    mfma_tile_step<true, true>(lds, tl, cur, nxt, nullptr, lam[t], eta, alpha);
}

// ---- int8 tiles of a batch: 64 replicas x 256 variables ---------------------------------
// For integer couplings with |J| <= 127 a workgroup owns 64 replicas (R0 .. R0 + 63) and
// 256 variables (I0 .. I0 + 255) of an instance; every tile row is a replica (with 64
// replicas per instance, as in the batch workload, no row is padding), and one tile does
// the work of two 128 x 128 tiles with one set of fixed costs.  Per chunk of 128 reduction
// variables a stage holds the 256 x 128 int8 block of J (rows of 128 bytes, the 16-byte
// piece p of row r at position p ^ (r % 8)) and the 64 x 128 byte spins of the tile's
// replicas (same layout); NST8 = 4 stages.
//   * matrix waves: wave w takes columns 64 (w % 4) .. + 63 and k steps 2 (w / 4),
//     2 (w / 4) + 1 of every chunk (32 each), 2 x 2 accumulators of 32 x 32
//     (v_mfma_i32_32x32x32_i8); they load the spins of every stage (one 1 KiB direct
//     load each: rows 8w .. 8w + 7) and, for dense rows, the couplings (four: rows
//     32w .. 32w + 31);
//   * state waves: thread t owns column t % 256 of rows 2e + t / 256 (32 rows); for
//     entry-list tiles, state wave g also writes the couplings of row groups 2g and 2g + 1
//     (16 rows each) of every stage: it clears their 2 KiB and stores each entry's weight
//     byte at its position (entries of chunk c placed after the barrier of chunk c - 2
//     into the stage of chunk c - 4, loaded three chunks ahead into three register sets
//     used in turn; lanes past a block's end repeat its last entry, the same byte with the
//     same value, so that no load or store sits behind a per-lane branch and each wait
//     for a register set covers that set only).
// After the reduction the two k halves' exact int32 partial sums go through two LDS
// buffers (rows padded to 264 words), added by the state waves, which then run the PA
// update and store x, m and the byte spins of their live rows (rows at or past rlive,
// uniform per wave, are skipped).  Barriers per tile: nchunk + 2 in both roles.

// The table's pointers are generic; these views make the offsets scalar loads (uniform,
// read-only during the launch) and the entries global loads, which count on the
// vector-memory counter only (generic loads also count on the counter that the LDS
// barriers wait for).
typedef __attribute__((address_space(4))) const int32_t c_i32;
typedef __attribute__((address_space(1))) const uint32_t g_u32;
typedef __attribute__((address_space(1))) const float g_f32;
typedef __attribute__((address_space(1))) float g_f32w;
typedef __attribute__((address_space(1))) uint8_t g_u8w;

// The LDS stores of this wave are complete, then the workgroup barrier.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <bool SPARSE>
__device__ __forceinline__ void matrix_tile8(uint8_t *lds, const Tile &tl, int nchunk,
                                             const uint8_t *__restrict__ s_cur, int wave,
                                             int lane) {
    const int64_t np = tl.np;
    const int kh = wave >> 2, wc = wave & 3;
    const int half = lane >> 5, l32 = lane & 31;
    // wave-uniform bases plus 32-bit lane offsets (fewer registers than 64-bit pointers):
    // load u of the couplings fills rows 32w + 8u + lane / 8, that of the spins rows
    // 8w + lane / 8, each at position lane % 8 (piece (lane % 8) ^ (row % 8))
    const uint8_t *Jw = reinterpret_cast<const uint8_t *>(tl.Jb) + (tl.I0 + 32 * wave) * np;
    const uint8_t *Sw = s_cur + (tl.R0 + 8 * wave) * KC;
    const int r8 = lane >> 3;
    const uint32_t piece = (uint32_t)((lane & 7) ^ r8);
    uint32_t oJ[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) oJ[u] = (uint32_t)(8 * u + r8) * (uint32_t)np + 16u * piece;
    const uint32_t oS = (uint32_t)r8 * (uint32_t)KC + 16u * piece;
    const int64_t sstride = tl.Rp * KC;            // bytes between consecutive spin chunks
    auto stage = [&](int kc, int st) {
        kc = kc < nchunk ? kc : nchunk - 1;        // past the end: reload the last chunk
        uint8_t *dst = lds + st * STG8;
        if (!SPARSE) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                __builtin_amdgcn_global_load_lds(Jw + (int64_t)kc * KC + oJ[u],
                                                 (lds_void *)(dst + (4 * wave + u) * 1024), 16, 0,
                                                 0);
        }
        __builtin_amdgcn_global_load_lds(Sw + (int64_t)kc * sstride + oS,
                                         (lds_void *)(dst + JSTG8 + wave * 1024), 16, 0, 0);
    };
    constexpr int LOADS = SPARSE ? 1 : 5;          // per chunk and wave
    i32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0;
#pragma unroll
    for (int s = 0; s < NST8 - 1; ++s) stage(s, s);
    for (int c = 0; c < nchunk; ++c) {
        // this wave's loads of chunk c have landed (NST8 - 2 younger chunks may not)
        wait_barrier<(NST8 - 2) * LOADS>();
        stage(c + NST8 - 1, (c + NST8 - 1) % NST8);
        const uint8_t *src = lds + (c % NST8) * STG8;
#pragma unroll
        for (int qq = 0; qq < 2; ++qq) {
            const int pc = 2 * (2 * kh + qq) + half;
            i32x4 a[2], bq[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int row = 32 * i + l32;
                a[i] = *reinterpret_cast<const i32x4 *>(src + JSTG8 + row * KC +
                                                        16 * (pc ^ (row & 7)));
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int row = 64 * wc + 32 * j + l32;
                bq[j] = *reinterpret_cast<const i32x4 *>(src + row * KC + 16 * (pc ^ (row & 7)));
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], bq[j], acc[i][j], 0,
                                                                      0, 0);
        }
    }
    wait_barrier<0>();     // every load has landed and every stage read is done
    // the two k halves' exact int32 partial sums, one buffer each
    int32_t *hp = reinterpret_cast<int32_t *>(lds) + kh * (BM8 * HS8);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = 32 * i + 8 * (v >> 2) + 4 * half + (v & 3);
                const int col = 64 * wc + 32 * j + l32;
                hp[row * HS8 + col] = acc[i][j][v];
            }
    wait_barrier<0>();     // partial sums stored
}

// Entries of one 16 x 128 block (I8S_EPL per lane).
struct EntryRegs {
    uint32_t e[I8S_EPL];
    int32_t cnt;
};

// Row group gg (0..15) of the tile, chunk kc (past the last chunk: the last again).  The
// block belongs to the 128-row tile I0 / 128 + gg / 8 of the entry-list layout.
__device__ __forceinline__ void entries_load(EntryRegs &er, const Tile &tl, int kc, int nchunk,
                                             int gg, int lane) {
    kc = kc < nchunk ? kc : nchunk - 1;
    const int64_t blk = ((tl.I0 / KC + (gg >> 3)) * (tl.np / KC) + kc) * 8 + (gg & 7);
    const c_i32 *O = (const c_i32 *)tl.O;
    const int32_t beg = O[blk];
    er.cnt = O[blk + 1] - beg;
    // an empty block reads the word at its start, which lies inside the coupling buffer
    // (the entries end at least a quarter of the buffer before its end); it is not placed
    // each block is read once per step and a batch's lists, state and spins are far more
    // than the caches hold between steps: non-temporal loads
    const g_u32 *src = (const g_u32 *)tl.E + beg;
    const int32_t last = max(er.cnt - 1, 0);
#pragma unroll
    for (int j = 0; j < I8S_EPL; ++j)
        er.e[j] = __builtin_nontemporal_load(&src[min(lane + 64 * j, last)]);
}

// Clears row group gg's 2 KiB of the stage and writes its entries there.  An entry's
// position within its 16 rows is its low 11 bits (the rows of its block); the words an
// empty block loaded write zeros into cleared bytes of the same rows.
__device__ __forceinline__ void entries_place(const EntryRegs &er, uint8_t *stage, int gg,
                                              int lane) {
    uint8_t *rg = stage + 2048 * gg;
    *reinterpret_cast<u32x4 *>(rg + 16 * lane) = (u32x4){0u, 0u, 0u, 0u};
    *reinterpret_cast<u32x4 *>(rg + 1024 + 16 * lane) = (u32x4){0u, 0u, 0u, 0u};
    const uint32_t keep = er.cnt > 0 ? 0xFFFFFFFFu : 0u;
#pragma unroll
    for (int j = 0; j < I8S_EPL; ++j)
        rg[er.e[j] & 0x7FFu] = (uint8_t)((er.e[j] & keep) >> 16);
}

// The two row groups (2g, 2g + 1) of a state wave.
struct EntryPair {
    EntryRegs a, b;
};

__device__ __forceinline__ void pair_load(EntryPair &p, const Tile &tl, int kc, int nchunk,
                                          int g, int lane) {
    entries_load(p.a, tl, kc, nchunk, 2 * g, lane);
    entries_load(p.b, tl, kc, nchunk, 2 * g + 1, lane);
}

__device__ __forceinline__ void pair_place(const EntryPair &p, uint8_t *stage, int g, int lane) {
    entries_place(p.a, stage, 2 * g, lane);
    entries_place(p.b, stage, 2 * g + 1, lane);
}

struct StateRegs8 {
    float xv[SR8], mv[SR8];
    float bi;
};

// x, m of rows 2e + t / 256, E0 <= e < E1, of this thread (rows at or past rlive are not
// read).  The state of a batch step (all instances', with the couplings and spins far more
// than the caches hold between steps) is read and written non-temporally.
template <int E0, int E1>
__device__ __forceinline__ void xm_load8(StateRegs8 &st, const Tile &tl, int t) {
    const int col = t & (BN8 - 1);
    const int rsub = __builtin_amdgcn_readfirstlane(t >> 8);
    const g_f32 *xr = (const g_f32 *)tl.x + (tl.R0 + 2 * E0 + rsub) * tl.np + tl.I0;
    const g_f32 *mr = (const g_f32 *)tl.m + (tl.R0 + 2 * E0 + rsub) * tl.np + tl.I0;
#pragma unroll
    for (int e = E0; e < E1; ++e) {
        const bool live = tl.R0 + 2 * e + rsub < tl.rlive;
        st.xv[e] = live ? __builtin_nontemporal_load(&xr[col]) : 0.0f;
        st.mv[e] = live ? __builtin_nontemporal_load(&mr[col]) : 0.0f;
        xr = next_rows(xr, 2 * tl.np);
        mr = next_rows(mr, 2 * tl.np);
    }
}

// One chunk barrier of a placing state wave: then the entries held in p (chunk c + 2) go
// into the stage of chunk c - 2 (free since the barrier of chunk c - 1) and p is reloaded
// with the chunk three further on.  Past the last chunk the reloaded last chunk is placed
// again, into a stage that no later chunk of the loop uses (they take those of c + 1 at
// most); the barrier after the loop waits for these stores.  No branch, so that the waits
// for one register set cover that set only.
__device__ __forceinline__ void place_step(EntryPair &p, const Tile &tl, int c, int nchunk,
                                           uint8_t *lds, int g, int lane) {
    lds_barrier();
    const int kc = c + NST8 - 2;
    pair_place(p, lds + (kc % NST8) * STG8, g, lane);
    pair_load(p, tl, kc + 3, nchunk, g, lane);
}

// State waves of an int8 tile, up to the partial sums: x, m and b loaded, and for
// entry-list tiles the couplings of every chunk placed.  Executes nchunk barriers.
template <bool SPARSE>
__device__ __forceinline__ void state_load8(StateRegs8 &st, const Tile &tl, int nchunk, int t,
                                            uint8_t *lds, int g, int lane) {
    static_assert(SR8 == 32 && NST8 == 4, "the load pattern below");
    const int col = t & (BN8 - 1);
    if (!SPARSE) {
        xm_load8<0, SR8>(st, tl, t);
        st.bi = ((const g_f32 *)tl.b)[tl.I0 + col];
        for (int c = 0; c < nchunk; ++c) barrier();
        return;
    }
    // the prologue's two chunks (past the last chunk: the last again, into stages no chunk
    // uses), then the next three chunks' entries; x and m follow in three groups after the
    // first three chunks' entry loads, since loads complete in issue order and a wait for
    // entries would otherwise wait for them
    EntryPair p0, p1, p2;
    pair_load(p0, tl, 0, nchunk, g, lane);
    pair_load(p1, tl, 1, nchunk, g, lane);
    pair_place(p0, lds, g, lane);
    pair_place(p1, lds + STG8, g, lane);
    pair_load(p0, tl, 2, nchunk, g, lane);
    pair_load(p1, tl, 3, nchunk, g, lane);
    pair_load(p2, tl, 4, nchunk, g, lane);
    if (nchunk > 0) place_step(p0, tl, 0, nchunk, lds, g, lane);
    xm_load8<0, 11>(st, tl, t);
    if (nchunk > 1) place_step(p1, tl, 1, nchunk, lds, g, lane);
    xm_load8<11, 22>(st, tl, t);
    if (nchunk > 2) place_step(p2, tl, 2, nchunk, lds, g, lane);
    xm_load8<22, 32>(st, tl, t);
    st.bi = ((const g_f32 *)tl.b)[tl.I0 + col];
    int c = 3;
    for (; c + 3 <= nchunk; c += 3) {
        place_step(p0, tl, c, nchunk, lds, g, lane);
        place_step(p1, tl, c + 1, nchunk, lds, g, lane);
        place_step(p2, tl, c + 2, nchunk, lds, g, lane);
    }
    if (c < nchunk) place_step(p0, tl, c, nchunk, lds, g, lane);
    if (c + 1 < nchunk) place_step(p1, tl, c + 1, nchunk, lds, g, lane);
}

// One PA step of one int8 tile.
template <bool SPARSE>
__device__ __forceinline__ void tile8_step(uint8_t *lds, const Tile &tl,
                                           const uint8_t *__restrict__ s_cur,
                                           uint8_t *__restrict__ s_nxt, float lt, float eta,
                                           float alpha) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nchunk = (int)(tl.np / KC);
    if (wave < MW) {
        matrix_tile8<SPARSE>(lds, tl, nchunk, s_cur, wave, lane);
        return;
    }
    const int t = tid - MW * 64;
    const int col = t & (BN8 - 1);
    const int rsub = __builtin_amdgcn_readfirstlane(t >> 8);
    StateRegs8 st;
    state_load8<SPARSE>(st, tl, nchunk, t, lds, wave - MW, lane);
    lds_barrier();                                     // stages drained (and written)
    barrier();                                         // partial sums stored
#pragma unroll
    for (int e = 0; e < SR8; ++e) asm volatile("" ::"v"(st.xv[e]), "v"(st.mv[e]));
    asm volatile("" ::"v"(st.bi));
    // field = sum of the two k halves' int32 partials (exact), unscaled; rows at or past
    // rlive (uniform per wave) are not read, not updated and their spins not written
    const int32_t *h0 = reinterpret_cast<const int32_t *>(lds), *h1 = h0 + BM8 * HS8;
    // spins as bytes: row r of chunk (I0 + col) / 128 at (chunk * Rp + r) * 128 + col % 128
    g_u8w *srow = (g_u8w *)s_nxt + (((tl.I0 + col) / KC) * tl.Rp + tl.R0 + rsub) * KC +
                  (col & (KC - 1));
    g_f32w *xr = (g_f32w *)tl.x + (tl.R0 + rsub) * tl.np + tl.I0 + col;
    g_f32w *mr = (g_f32w *)tl.m + (tl.R0 + rsub) * tl.np + tl.I0 + col;
#pragma unroll
    for (int g = 0; g < SR8 / 8; ++g) {
        if (tl.R0 + 2 * (8 * g) + rsub >= tl.rlive) continue;
        int32_t hv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = (2 * (8 * g + u) + rsub) * HS8 + col;
            hv[u] = h0[k] + h1[k];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = 8 * g + u;
            if (tl.R0 + 2 * e + rsub < tl.rlive) {
                const float h = __fadd_rn((float)hv[u], st.bi);
                pa_update(h, lt, eta, alpha, st.xv[e], st.mv[e]);
                srow[(int64_t)2 * e * KC] = st.xv[e] < 0.0f ? (uint8_t)0xFF : (uint8_t)0x01;
                __builtin_nontemporal_store(st.xv[e], &xr[(int64_t)2 * e * tl.np]);
                __builtin_nontemporal_store(st.mv[e], &mr[(int64_t)2 * e * tl.np]);
            }
        }
    }
}

template <bool SPARSE>
__global__ void __launch_bounds__(THREADS, 1) k_mfma_grouped8(const MfmaTile *__restrict__ tiles,
                                                              int t, const float *__restrict__ lam,
                                                              float eta, float alpha) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[LDS_BYTES];
    const MfmaTile mt = tiles[blockIdx.x];
    if (mt.np == 0) return;      // filler entry of the compute-die-ordered table
    const uint8_t *cur = reinterpret_cast<const uint8_t *>((t & 1) ? mt.s1 : mt.s0);
    uint8_t *nxt = reinterpret_cast<uint8_t *>((t & 1) ? mt.s0 : mt.s1);
    const Tile tl{mt.np, mt.Rp, mt.I0, mt.R0, mt.rlive, mt.Jb, mt.b, 1.0f, mt.x, mt.m,
                  mt.E, mt.O};
    tile8_step<SPARSE>(lds, tl, cur, nxt, lam[t], eta, alpha);
}

// Byte spins of the signs of x (chunk-major, 128 bytes per replica and chunk).
__global__ void __launch_bounds__(256) k_mfma_pack_i8(int64_t Rp, int64_t np,
                                                      const float *__restrict__ x,
                                                      uint8_t *__restrict__ s8) {
    const int64_t total = Rp * np;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t kc = k / (Rp * KC), rem = k - kc * Rp * KC;
        const int64_t r = rem / KC, j = rem - r * KC;
        s8[k] = x[r * np + KC * kc + j] < 0.0f ? (uint8_t)0xFF : (uint8_t)0x01;
    }
}

// Pair words of the signs of x (layout above): one thread per word.
__global__ void __launch_bounds__(256) k_mfma_pack(int64_t Rp, int64_t np,
                                                   const float *__restrict__ x,
                                                   uint32_t *__restrict__ sw) {
    const int64_t total = Rp * (np / 8);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t kc = k / (Rp * 16), rem = k - kc * Rp * 16;
        const int64_t r = rem / 16, wd = rem - r * 16;
        const int64_t h = wd >> 3, q = wd & 7;
        const float *xr = x + r * np + KC * kc + 16 * q + 8 * h;
        uint32_t byte = 0;
        for (int j = 0; j < 8; ++j) byte |= (xr[j] < 0.0f ? 1u : 0u) << j;
        sw[k] = spin_pair(byte);
    }
}

// ---- sparse int8 tiles: entry lists of the 16 x 128 blocks of J8 ------------------------
// One wave per block: lane l covers row 16 g + l / 4 of the row tile, columns
// 32 (l % 4) .. 32 (l % 4) + 31 of the chunk.
__device__ __forceinline__ void i8s_block(const I8sTask &tk, int64_t blk, int lane,
                                          const int8_t *&src, int &row, int &k0) {
    const int64_t nch = tk.np / KC;
    const int64_t ib = blk / (nch * 8), kc = (blk / 8) % nch, g = blk % 8;
    row = 16 * (int)g + (lane >> 2);
    k0 = 32 * (lane & 3);
    src = tk.J8 + (ib * KC + row) * tk.np + kc * KC + k0;
}

__device__ __forceinline__ int nonzero_bytes(uint32_t v) {
    int c = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) c += ((v >> (8 * b)) & 0xFFu) != 0u;
    return c;
}

__global__ void __launch_bounds__(256) k_i8s_count(const I8sTask *__restrict__ tasks) {
    const I8sTask tk = tasks[blockIdx.y];
    const int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (blk >= i8s_blocks(tk.np)) return;                 // whole waves leave together
    const int8_t *src;
    int row, k0;
    i8s_block(tk, blk, lane, src, row, k0);
    const u32x4 v0 = *reinterpret_cast<const u32x4 *>(src);
    const u32x4 v1 = *reinterpret_cast<const u32x4 *>(src + 16);
    int c = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) c += nonzero_bytes(v0[q]) + nonzero_bytes(v1[q]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (lane == 0) tk.cnt[blk] = c;
}

// Counts -> exclusive offsets in place (nblk + 1 values, the last the total), and the
// largest block and the total into stats.  One workgroup per task.
__global__ void __launch_bounds__(1024) k_i8s_scan(const I8sTask *__restrict__ tasks) {
    __shared__ int32_t part[1024], mx[1024];
    const I8sTask tk = tasks[blockIdx.x];
    const int64_t nblk = i8s_blocks(tk.np);
    const int t = threadIdx.x;
    const int64_t per = (nblk + 1023) / 1024;
    const int64_t a = std::min<int64_t>(nblk, t * per), b = std::min<int64_t>(nblk, a + per);
    int32_t s = 0, m = 0;
    for (int64_t i = a; i < b; ++i) {
        s += tk.cnt[i];
        m = max(m, tk.cnt[i]);
    }
    part[t] = s;
    mx[t] = m;
    __syncthreads();
    if (t == 0) {                 // 1024 partial sums in order: exact and deterministic
        int32_t run = 0, mm = 0;
        for (int i = 0; i < 1024; ++i) {
            const int32_t v = part[i];
            part[i] = run;
            run += v;
            mm = max(mm, mx[i]);
        }
        tk.stats[0] = mm;
        tk.stats[1] = run;
        tk.cnt[nblk] = run;
    }
    __syncthreads();
    int32_t run = part[t];
    for (int64_t i = a; i < b; ++i) {
        const int32_t v = tk.cnt[i];
        tk.cnt[i] = run;
        run += v;
    }
}

// The entries of every block (tasks whose largest block exceeds I8S_BLOCK_MAX keep their
// dense rows and are skipped).  Within a block the entries follow (row, column) order.
__global__ void __launch_bounds__(256) k_i8s_fill(const I8sTask *__restrict__ tasks) {
    const I8sTask tk = tasks[blockIdx.y];
    const int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (blk >= i8s_blocks(tk.np) || tk.stats[0] > I8S_BLOCK_MAX) return;
    const int8_t *src;
    int row, k0;
    i8s_block(tk, blk, lane, src, row, k0);
    const u32x4 v0 = *reinterpret_cast<const u32x4 *>(src);
    const u32x4 v1 = *reinterpret_cast<const u32x4 *>(src + 16);
    int c = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) c += nonzero_bytes(v0[q]) + nonzero_bytes(v1[q]);
    int incl = c;                                     // inclusive prefix over the lanes
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    uint32_t *dst = tk.E + tk.cnt[blk] + (incl - c);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const uint32_t v = q < 4 ? v0[q] : v1[q - 4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t w = (v >> (8 * b)) & 0xFFu;
            if (w != 0u) {
                const int k = k0 + 4 * q + b;
                const uint32_t pos = (uint32_t)(row * KC + 16 * ((k >> 4) ^ (row & 7)) + (k & 15));
                *dst++ = (w << 16) | pos;
            }
        }
    }
}

}  // namespace

hipError_t launch_i8s_count(const I8sTask *tasks, int32_t ntask, int64_t max_np,
                            hipStream_t st) {
    if (ntask <= 0) return hipSuccess;
    const int64_t bx = (i8s_blocks(max_np) + 3) / 4;
    if (bx <= 0 || bx > INT32_MAX || ntask > 65535) return hipErrorInvalidValue;
    k_i8s_count<<<dim3((unsigned)bx, (unsigned)ntask), 256, 0, st>>>(tasks);
    return hipGetLastError();
}

hipError_t launch_i8s_scan(const I8sTask *tasks, int32_t ntask, hipStream_t st) {
    if (ntask <= 0) return hipSuccess;
    k_i8s_scan<<<(unsigned)ntask, 1024, 0, st>>>(tasks);
    return hipGetLastError();
}

hipError_t launch_i8s_fill(const I8sTask *tasks, int32_t ntask, int64_t max_np,
                           hipStream_t st) {
    if (ntask <= 0) return hipSuccess;
    const int64_t bx = (i8s_blocks(max_np) + 3) / 4;
    if (bx <= 0 || bx > INT32_MAX || ntask > 65535) return hipErrorInvalidValue;
    k_i8s_fill<<<dim3((unsigned)bx, (unsigned)ntask), 256, 0, st>>>(tasks);
    return hipGetLastError();
}

hipError_t launch_mfma_pack_spins(int64_t Rp, int64_t np, const float *x, uint32_t *sbits,
                                  hipStream_t st) {
    int64_t total = Rp * (np / 8);
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
                               const float *lam, float eta, float alpha, GroupKind kind,
                               hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (kind == GK_I8_SPARSE)
        k_mfma_grouped8<true><<<(unsigned)ntiles, THREADS, 0, st>>>(tiles, t, lam, eta, alpha);
    else if (kind == GK_I8)
        k_mfma_grouped8<false><<<(unsigned)ntiles, THREADS, 0, st>>>(tiles, t, lam, eta, alpha);
    else
        k_mfma_grouped<<<(unsigned)ntiles, THREADS, 0, st>>>(tiles, t, lam, eta, alpha);
    return hipGetLastError();
}

hipError_t launch_mfma_pack_spins_i8(int64_t Rp, int64_t np, const float *x, uint8_t *s8,
                                     hipStream_t st) {
    int64_t g = (Rp * np + 255) / 256;
    if (g > 65536) g = 65536;
    k_mfma_pack_i8<<<(unsigned)g, 256, 0, st>>>(Rp, np, x, s8);
    return hipGetLastError();
}

// Dense int8 copy of a CSR instance (integer weights with |w| <= 127, checked by the
// caller): J8[i][j] = w_ij for the stored off-diagonal entries, zero elsewhere (the caller
// clears J8 first).  One wave per row.
template <typename TW, typename TI>
__global__ void __launch_bounds__(256) k_csr_to_i8(int64_t n, int64_t np,
                                                   const int32_t *__restrict__ rp,
                                                   const TI *__restrict__ col,
                                                   const TW *__restrict__ w,
                                                   int8_t *__restrict__ J8) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += 64) {
        const int64_t j = (int64_t)col[k];
        if (j == i) continue;
        J8[i * np + j] = (int8_t)w[k];
    }
}

// The same matrix written whole, one workgroup per row (rows n .. np-1 zero): the row is
// cleared and its entries placed in LDS, then stored in 16-byte pieces, so that the
// matrix needs no separate clear.  np is a multiple of 128 and at most ROWS8_MAX_NP.
constexpr int64_t ROWS8_MAX_NP = 65536;

template <typename TW, typename TI>
__device__ __forceinline__ void csr_to_i8_row(int64_t i, int64_t n, int64_t np,
                                              const int32_t *__restrict__ rp,
                                              const TI *__restrict__ col,
                                              const TW *__restrict__ w,
                                              int8_t *__restrict__ J8) {
    extern __shared__ uint4 row16[];              // np bytes
    int8_t *row = reinterpret_cast<int8_t *>(row16);
    const int64_t np16 = np / 16;
    for (int64_t q = threadIdx.x; q < np16; q += blockDim.x) row16[q] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    if (i < n) {
        for (int64_t k = rp[i] + threadIdx.x; k < rp[i + 1]; k += blockDim.x) {
            const int64_t j = (int64_t)col[k];
            if (j != i) row[j] = (int8_t)w[k];
        }
    }
    __syncthreads();
    uint4 *dst = reinterpret_cast<uint4 *>(J8 + i * np);
    for (int64_t q = threadIdx.x; q < np16; q += blockDim.x) dst[q] = row16[q];
}

template <typename TW, typename TI>
__global__ void __launch_bounds__(256) k_csr_to_i8_rows(int64_t n, int64_t np,
                                                        const int32_t *__restrict__ rp,
                                                        const TI *__restrict__ col,
                                                        const TW *__restrict__ w,
                                                        int8_t *__restrict__ J8) {
    csr_to_i8_row<TW, TI>(blockIdx.x, n, np, rp, col, w, J8);
}

// Batched: row blockIdx.x of instance blockIdx.y (rows past the instance's np return).
template <typename TW, typename TI>
__global__ void __launch_bounds__(256) k_csr_to_i8_rows_batch(const SlotInitTask *__restrict__ tasks) {
    const SlotInitTask &t = tasks[blockIdx.y];
    if ((int64_t)blockIdx.x >= t.np) return;
    csr_to_i8_row<TW, TI>(blockIdx.x, t.n, t.np, t.rp, static_cast<const TI *>(t.col),
                          static_cast<const TW *>(t.w), t.J8);
}

hipError_t launch_csr_to_i8_batch(const SlotInitTask *tasks, int32_t ntask, qpa_dtype coupling,
                                  qpa_dtype index, int64_t max_np, hipStream_t st) {
    if (max_np < MF_NPAD || max_np % MF_NPAD || max_np > ROWS8_MAX_NP)
        return hipErrorInvalidValue;
    auto run = [&](auto wtag, auto itag) {
        using TW = decltype(wtag);
        using TI = decltype(itag);
        for (int32_t c0 = 0; c0 < ntask; c0 += 65535) {
            const dim3 g((unsigned)max_np, (unsigned)std::min(65535, ntask - c0));
            k_csr_to_i8_rows_batch<TW, TI><<<g, 256, (size_t)max_np, st>>>(tasks + c0);
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

hipError_t launch_csr_to_i8(const qpa_problem &p, int64_t np, int8_t *J8, hipStream_t st) {
    const bool rows = np % 128 == 0 && np >= p.n && np <= ROWS8_MAX_NP;
    if (!rows) {
        const hipError_t e = hipMemsetAsync(J8, 0, (size_t)(np * np), st);
        if (e != hipSuccess) return e;
    }
    const int64_t g = (p.n + 3) / 4;
    auto run = [&](auto wtag, auto itag) {
        using TW = decltype(wtag);
        using TI = decltype(itag);
        if (rows)
            k_csr_to_i8_rows<TW, TI><<<(unsigned)np, 256, (size_t)np, st>>>(
                p.n, np, p.row_ptr, static_cast<const TI *>(p.col),
                static_cast<const TW *>(p.weights), J8);
        else
            k_csr_to_i8<TW, TI><<<(unsigned)g, 256, 0, st>>>(
                p.n, np, p.row_ptr, static_cast<const TI *>(p.col),
                static_cast<const TW *>(p.weights), J8);
        return hipGetLastError();
    };
    auto byw = [&](auto itag) -> hipError_t {
        switch (p.coupling_dtype) {
            case QPA_I8: return run((int8_t)0, itag);
            case QPA_I16: return run((int16_t)0, itag);
            case QPA_I32: return run((int32_t)0, itag);
            default: return hipErrorInvalidValue;
        }
    };
    return p.index_dtype == QPA_I16 ? byw((int16_t)0) : byw((int32_t)0);
}


// Dense BF16 copy of a CSR instance: Jb[i][j] = bf16(w_ij * 2^-e) for the stored
// off-diagonal entries (zero elsewhere; the caller clears Jb first).  One wave per row,
// the row's entries split over the lanes.
template <typename TW, typename TI>
__global__ void __launch_bounds__(256) k_csr_to_bf16(int64_t n, int64_t np,
                                                     const int32_t *__restrict__ rp,
                                                     const TI *__restrict__ col,
                                                     const TW *__restrict__ w,
                                                     const CanonScalars *__restrict__ sc,
                                                     uint16_t *__restrict__ Jb) {
    const float inv = sc->inv_scale;
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += 64) {
        const int64_t j = (int64_t)col[k];
        if (j == i) continue;
        uint32_t u = __float_as_uint(__fmul_rn((float)w[k], inv));
        u += 0x7fffu + ((u >> 16) & 1u);
        Jb[i * np + j] = (uint16_t)(u >> 16);
    }
}

hipError_t launch_csr_to_bf16(const qpa_problem &p, int64_t np, const CanonScalars *sc,
                              uint16_t *Jb, hipStream_t st) {
    hipError_t e = hipMemsetAsync(Jb, 0, sizeof(uint16_t) * (size_t)(np * np), st);
    if (e != hipSuccess) return e;
    const int64_t g = (p.n + 3) / 4;
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
