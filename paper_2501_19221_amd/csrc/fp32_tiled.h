// LDS-tiled FP32 product on the vector units, shared by the SBM step, the PA FP32 dense
// step and the relaxed-dynamics adjoint:  G = J Q  with J [n][n] symmetric (row k of J
// is column k) and Q [n][Rp] (replica fastest), followed by a per-tile epilogue.
//
// A workgroup owns a 128 (replicas) x 128 (variables) output tile; each of its 256
// threads holds 8 x 8 sums and adds one term per reduction index with a fused
// multiply-add, in ascending order.  Chunks of 32 reduction indices of Q and J are
// double-buffered in LDS; the next chunk is prefetched into registers while the current
// one is multiplied.  The epilogue receives the tile's sums: thread (tx, ty) holds
// replicas r0 + 64h + 4ty + e (h < 2, e < 4) and variables i0 + 64(v/4) + 4tx + v%4.
#pragma once

#include "qpa_internal.h"

namespace qpa {
namespace {

constexpr int SB_BR = 128;   // replicas per dense tile
constexpr int SB_BI = 128;   // variables per dense tile
constexpr int SB_KC = 32;    // reduction indices per LDS chunk

__device__ __forceinline__ float4 sb_load_q(const float *__restrict__ qi, int64_t k, int64_t n,
                                           int64_t Rp, int64_t col) {
    if (k < n) return *reinterpret_cast<const float4 *>(qi + k * Rp + col);
    // past the last row: -0.0 times the padding's zero couplings is exactly -0.0, which
    // leaves every sum unchanged (also a -0.0 left by an underflowing product)
    return make_float4(-0.0f, -0.0f, -0.0f, -0.0f);
}

// VEC: n % 4 == 0, so rows of J can be read as float4.
template <bool VEC>
__device__ __forceinline__ float4 sb_load_j(const float *__restrict__ J, int64_t k, int64_t n,
                                           int64_t i) {
    float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (k >= n) return v;
    const float *row = J + k * n;
    if (VEC) {
        if (i < n) v = *reinterpret_cast<const float4 *>(row + i);
    } else {
        if (i < n) v.x = row[i];
        if (i + 1 < n) v.y = row[i + 1];
        if (i + 2 < n) v.z = row[i + 2];
        if (i + 3 < n) v.w = row[i + 3];
    }
    return v;
}

typedef __attribute__((address_space(3))) const void sb_lds_t;
typedef float sb_f4 __attribute__((ext_vector_type(4)));

// LDS byte address of a shared-memory pointer.
__device__ __forceinline__ uint32_t sb_lds(const float4 *p) {
    return (uint32_t)(uintptr_t)(sb_lds_t *)p;
}

// Issue the four fragment reads of one reduction index: A columns at la + off and
// la + off + 256 (replicas 4ty.. and 64+4ty..), B at lb + off and lb + off + 256.
__device__ __forceinline__ void sb_rd4(sb_f4 &a0, sb_f4 &a1, sb_f4 &b0, sb_f4 &b1,
                                       uint32_t la, uint32_t lb, int off_tag) {
    if (off_tag == 0) {
        asm volatile("ds_read_b128 %0, %4\n\tds_read_b128 %1, %4 offset:256\n\t"
                     "ds_read_b128 %2, %5\n\tds_read_b128 %3, %5 offset:256"
                     : "=v"(a0), "=v"(a1), "=v"(b0), "=v"(b1) : "v"(la), "v"(lb));
    } else if (off_tag == 512) {
        asm volatile("ds_read_b128 %0, %4 offset:512\n\tds_read_b128 %1, %4 offset:768\n\t"
                     "ds_read_b128 %2, %5 offset:512\n\tds_read_b128 %3, %5 offset:768"
                     : "=v"(a0), "=v"(a1), "=v"(b0), "=v"(b1) : "v"(la), "v"(lb));
    } else {
        asm volatile("ds_read_b128 %0, %4 offset:1024\n\tds_read_b128 %1, %4 offset:1280\n\t"
                     "ds_read_b128 %2, %5 offset:1024\n\tds_read_b128 %3, %5 offset:1280"
                     : "=v"(a0), "=v"(a1), "=v"(b0), "=v"(b1) : "v"(la), "v"(lb));
    }
}

// Wait until at most N LDS reads of this wave are outstanding; the registers are tied to
// the wait so that no use is scheduled before it.
template <int N>
__device__ __forceinline__ void sb_wait4(sb_f4 &a0, sb_f4 &a1, sb_f4 &b0, sb_f4 &b1) {
    asm volatile("s_waitcnt lgkmcnt(%4)" : "+v"(a0), "+v"(a1), "+v"(b0), "+v"(b1) : "n"(N));
}

#define SB_FMA_ROW(u, av)                                                               \
    acc[u][0] = __fmaf_rn(av, fb0.x, acc[u][0]);                                         \
    acc[u][1] = __fmaf_rn(av, fb0.y, acc[u][1]);                                         \
    acc[u][2] = __fmaf_rn(av, fb0.z, acc[u][2]);                                         \
    acc[u][3] = __fmaf_rn(av, fb0.w, acc[u][3]);                                         \
    acc[u][4] = __fmaf_rn(av, fb1.x, acc[u][4]);                                         \
    acc[u][5] = __fmaf_rn(av, fb1.y, acc[u][5]);                                         \
    acc[u][6] = __fmaf_rn(av, fb1.z, acc[u][6]);                                         \
    acc[u][7] = __fmaf_rn(av, fb1.w, acc[u][7]);

// FP32 tiled product G = J Q ([n][n] x [n][Rp], both read row by row: J is symmetric, so
// its row k is column k) with a per-step epilogue: the SBM step (Q = positions) or the PA
// step (Q = spins as +-1 floats).
template <bool VEC, class Epi>
__global__ void __launch_bounds__(256) k_fp32_tiled_step(int64_t n, int64_t Rp,
                                                         const float *__restrict__ J,
                                                         const float *__restrict__ qi,
                                                         const Epi epi) {
    __shared__ float4 As[2][SB_KC + 1][SB_BR / 4];
    __shared__ float4 Bs[2][SB_KC + 1][SB_BI / 4];
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const int64_t i0 = (int64_t)blockIdx.x * SB_BI, r0 = (int64_t)blockIdx.y * SB_BR;
    float acc[8][8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int v = 0; v < 8; ++v) acc[u][v] = 0.0f;
    // load slots of this thread in a chunk: rows kk = t/32 + 8e (e < 4), float4 column t%32
    const int lk = t >> 5, lc = t & 31;
    const int64_t qcol = r0 + 4 * lc, jcol = i0 + 4 * lc;
    float4 pa0, pa1, pa2, pa3, pb0, pb1, pb2, pb3;
#define SB_FETCH(k0)                                                                     \
    pa0 = sb_load_q(qi, (k0) + lk, n, Rp, qcol);                                         \
    pa1 = sb_load_q(qi, (k0) + lk + 8, n, Rp, qcol);                                     \
    pa2 = sb_load_q(qi, (k0) + lk + 16, n, Rp, qcol);                                    \
    pa3 = sb_load_q(qi, (k0) + lk + 24, n, Rp, qcol);                                    \
    pb0 = sb_load_j<VEC>(J, (k0) + lk, n, jcol);                                         \
    pb1 = sb_load_j<VEC>(J, (k0) + lk + 8, n, jcol);                                     \
    pb2 = sb_load_j<VEC>(J, (k0) + lk + 16, n, jcol);                                    \
    pb3 = sb_load_j<VEC>(J, (k0) + lk + 24, n, jcol);
#define SB_STASH(buf)                                                                    \
    As[buf][lk][lc] = pa0;                                                               \
    As[buf][lk + 8][lc] = pa1;                                                           \
    As[buf][lk + 16][lc] = pa2;                                                          \
    As[buf][lk + 24][lc] = pa3;                                                          \
    Bs[buf][lk][lc] = pb0;                                                               \
    Bs[buf][lk + 8][lc] = pb1;                                                           \
    Bs[buf][lk + 16][lc] = pb2;                                                          \
    Bs[buf][lk + 24][lc] = pb3;
    const int64_t nch = (n + SB_KC - 1) / SB_KC;
    SB_FETCH(0)
    SB_STASH(0)
    __syncthreads();
    for (int64_t c = 0; c < nch; ++c) {
        const int buf = (int)(c & 1);
        const bool more = c + 1 < nch;
        if (more) {
            SB_FETCH((c + 1) * SB_KC)
        }
        // Two fragment sets: while one reduction index is multiplied, the next one's
        // fragments are read.  The reads are issued by inline assembly (the compiler would
        // otherwise move them next to their use) and their completion is awaited by
        // explicit waits that also mark the registers as written.  Row SB_KC of each
        // buffer is padding: read, never used.
        const uint32_t la = sb_lds(&As[buf][0][ty]), lb = sb_lds(&Bs[buf][0][tx]);
        sb_f4 xa0, xa1, xb0, xb1, ya0, ya1, yb0, yb1;
        sb_rd4(xa0, xa1, xb0, xb1, la, lb, 0);
#pragma unroll 1
        for (int kk = 0; kk < SB_KC; kk += 2) {
            const uint32_t o = (uint32_t)kk * 512u;
            sb_rd4(ya0, ya1, yb0, yb1, la + o, lb + o, 512);
            sb_wait4<4>(xa0, xa1, xb0, xb1);
            {
                const sb_f4 fb0 = xb0, fb1 = xb1;
                SB_FMA_ROW(0, xa0.x)
                SB_FMA_ROW(1, xa0.y)
                SB_FMA_ROW(2, xa0.z)
                SB_FMA_ROW(3, xa0.w)
                SB_FMA_ROW(4, xa1.x)
                SB_FMA_ROW(5, xa1.y)
                SB_FMA_ROW(6, xa1.z)
                SB_FMA_ROW(7, xa1.w)
            }
            sb_rd4(xa0, xa1, xb0, xb1, la + o, lb + o, 1024);
            sb_wait4<4>(ya0, ya1, yb0, yb1);
            {
                const sb_f4 fb0 = yb0, fb1 = yb1;
                SB_FMA_ROW(0, ya0.x)
                SB_FMA_ROW(1, ya0.y)
                SB_FMA_ROW(2, ya0.z)
                SB_FMA_ROW(3, ya0.w)
                SB_FMA_ROW(4, ya1.x)
                SB_FMA_ROW(5, ya1.y)
                SB_FMA_ROW(6, ya1.z)
                SB_FMA_ROW(7, ya1.w)
            }
        }
        sb_wait4<0>(xa0, xa1, xb0, xb1);     // the padding row's reads land before reuse
        if (more) {
            SB_STASH(buf ^ 1)
        }
        __syncthreads();
    }
#undef SB_FETCH
#undef SB_STASH
    epi(acc, n, Rp, i0, r0, tx, ty);
}
#undef SB_FMA_ROW

}  // namespace
}  // namespace qpa
