// Binned sparse PA step (App. B field h = J s + b and the fused update) for CSR instances
// with integer couplings and at most 8 replicas.
//
// When the spin words of a large graph far exceed the L2 cache, the per-row gather of the
// streamed kernel pulls one cache line per coupling, about 16x the bytes of the CSR entry
// it serves.  Here the gather is split into two streaming passes over an entry order
// fixed once per run (propagation blocking):
//   source chunks: C = 2^20 / G variables, whose spin words (128 KiB) fit in LDS;
//   destination bins: B = 2^14 L / G rows, whose field sums fit in 2^14 words of LDS,
//     L = 4, 2 or 1 sums per word (8-, 16- or 32-bit lanes, chosen from the row bound);
//   entries (diagonal excluded for QUBO) ordered by (chunk, bin), any order inside a block.
//   pass 1, k_bin_gather: a workgroup loads the spin words of one chunk into LDS and, for
//     a contiguous share of the chunk's entries, writes the G spin bits of each entry's
//     column to bits[p];
//   pass 2, k_bin_update: a workgroup clears its sums in LDS and adds, for every entry of
//     its bin, |w| b' per replica with b' = b XOR [w < 0] (one LDS atomic per word of L
//     lanes); the field is then h = c - 2 A with A the replica's sum and c = sum |w| + b
//     per row (built once per call), since a term w (1 - 2b) equals |w| (1 - 2b').  Then
//     the fused update of its rows (x, m, spin words), the arithmetic of the streamed
//     kernel.  A lane of W bits never carries into the next: A <= sum |w| < 2^W.
// Integer sums are exact, so the order of the entries inside a block does not change a
// bit of the result, and (float)(c - 2A) equals the streamed kernel's (float)sum + b.
// Entries carry the column's offset in its chunk (uint32) and the row's offset in its bin
// with the weight (low / high 16 bits of a uint32).
#include "qpa_internal.h"

namespace qpa {
namespace {

constexpr int BT = 1024;                 // threads per workgroup of every kernel here
constexpr int CHUNK_WORDS = 1 << 14;     // spin words (uint64) of one source chunk
constexpr int BIN_WORDS = 1 << 14;       // LDS words of field sums of one bin
constexpr int SCAN_TILE = 4 * BT;        // elements per workgroup of the offset scan

__device__ __forceinline__ void pa_update(float h, float lam, float eta, float alpha, float &x,
                                          float &m) {
    float g = __fadd_rn(__fmul_rn(lam, x), h);
    float mn = __fsub_rn(__fmul_rn(alpha, m), __fmul_rn(eta, g));
    float y = __fadd_rn(x, mn);
    y = fminf(1.0f, fmaxf(-1.0f, y));
    m = mn;
    x = y;
}

// Exclusive prefix sums of PER values per thread over a 1024-thread workgroup, in thread
// order; returns the workgroup total.  `wsum` holds 16 ints of LDS.
template <int PER>
__device__ int32_t block_scan_excl(int32_t (&v)[PER], int32_t *wsum) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t own = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int32_t t = v[u];
        v[u] = own;
        own += t;
    }
    int32_t inc = own;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    int32_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < BT / 64; ++w) {
        const int32_t s = wsum[w];
        before += w < wave ? s : 0;
        total += s;
    }
    __syncthreads();
    const int32_t base = before + inc - own;
#pragma unroll
    for (int u = 0; u < PER; ++u) v[u] += base;
    return total;
}

__global__ void __launch_bounds__(256) k_bin_fill(int32_t *__restrict__ p, int64_t cnt) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < cnt;
         q += (int64_t)gridDim.x * blockDim.x)
        p[q] = 0;
}

// Entries per (chunk, bin) block.  Thread per row; columns were validated in range.
template <typename TI>
__global__ void __launch_bounds__(256) k_bin_count(int64_t n, const int32_t *__restrict__ rp,
                                                   const TI *__restrict__ col, int skip_diag,
                                                   int cshift, int bshift, int64_t Nb,
                                                   int32_t *__restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t bb = i >> bshift;
    const int32_t k1 = rp[i + 1];
    for (int32_t k = rp[i]; k < k1; ++k) {
        const int64_t j = (int64_t)col[k];
        if (skip_diag && j == i) continue;
        atomicAdd(&cnt[(j >> cshift) * Nb + bb], 1);
    }
}

// Offset scan, step 1: the total of every SCAN_TILE-element tile.
__global__ void __launch_bounds__(BT) k_bin_tile_sums(const int32_t *__restrict__ cnt, int64_t M,
                                                      int32_t *__restrict__ tsum) {
    __shared__ int32_t wsum[BT / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * 4;
    int32_t v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = base + u < M ? cnt[base + u] : 0;
    const int32_t tot = block_scan_excl<4>(v, wsum);
    if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

// Step 2 (one workgroup): exclusive scan of the tile totals in place; off[M] = total.
__global__ void __launch_bounds__(BT) k_bin_scan_tiles(int32_t *__restrict__ tsum, int64_t nt,
                                                       int32_t *__restrict__ off, int64_t M) {
    __shared__ int32_t wsum[BT / 64];
    int32_t carry = 0;
    for (int64_t b0 = 0; b0 < nt; b0 += SCAN_TILE) {
        const int64_t base = b0 + (int64_t)threadIdx.x * 4;
        int32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = base + u < nt ? tsum[base + u] : 0;
        const int32_t tot = block_scan_excl<4>(v, wsum);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (base + u < nt) tsum[base + u] = v[u] + carry;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) off[M] = carry;
}

// Step 3: exclusive offsets of every block, and a copy used as the scatter cursor.
__global__ void __launch_bounds__(BT) k_bin_offsets(const int32_t *__restrict__ cnt, int64_t M,
                                                    const int32_t *__restrict__ tsum,
                                                    int32_t *__restrict__ off,
                                                    int32_t *__restrict__ cur) {
    __shared__ int32_t wsum[BT / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * 4;
    int32_t v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = base + u < M ? cnt[base + u] : 0;
    (void)block_scan_excl<4>(v, wsum);
    const int32_t t0 = tsum[blockIdx.x];
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (base + u < M) {
            off[base + u] = v[u] + t0;
            cur[base + u] = v[u] + t0;
        }
}

// Entries into their blocks: column offset in its chunk, row offset in its bin | weight.
template <typename TI, typename TW>
__global__ void __launch_bounds__(256) k_bin_scatter(int64_t n, const int32_t *__restrict__ rp,
                                                     const TI *__restrict__ col,
                                                     const TW *__restrict__ w, int skip_diag,
                                                     int cshift, int bshift, int64_t Nb,
                                                     int32_t *__restrict__ cur,
                                                     uint32_t *__restrict__ src,
                                                     uint32_t *__restrict__ drec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t bb = i >> bshift;
    const uint32_t dl = (uint32_t)(i & ((1ll << bshift) - 1));
    const uint32_t cmask = (uint32_t)((1ll << cshift) - 1);
    const int32_t k1 = rp[i + 1];
    for (int32_t k = rp[i]; k < k1; ++k) {
        const int64_t j = (int64_t)col[k];
        if (skip_diag && j == i) continue;
        const int32_t pos = atomicAdd(&cur[(j >> cshift) * Nb + bb], 1);
        src[pos] = (uint32_t)j & cmask;
        drec[pos] = dl | ((uint32_t)(uint16_t)(int16_t)w[k] << 16);
    }
}

// Row constants c_i = sum over off-diagonal entries of |w| + b_i (exact integers).
template <typename TI, typename TW>
__global__ void __launch_bounds__(256) k_bin_rowconst(int64_t n, const int32_t *__restrict__ rp,
                                                      const TI *__restrict__ col,
                                                      const TW *__restrict__ w, int skip_diag,
                                                      const int64_t *__restrict__ b_i64,
                                                      int32_t *__restrict__ crow) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t c = b_i64[i];
    const int32_t k1 = rp[i + 1];
    for (int32_t k = rp[i]; k < k1; ++k) {
        if (skip_diag && (int64_t)col[k] == i) continue;
        const int64_t v = (int64_t)w[k];
        c += v < 0 ? -v : v;
    }
    crow[i] = (int32_t)c;
}

// Pass 1.  Grid (Nc, S): chunk c, share s of its entries.
__global__ void __launch_bounds__(BT) k_bin_gather(int shiftG, int64_t nwords, int64_t Nb,
                                                   const int32_t *__restrict__ off,
                                                   const uint32_t *__restrict__ src,
                                                   const uint64_t *__restrict__ s_cur,
                                                   uint8_t *__restrict__ bits) {
    __shared__ uint64_t words[CHUNK_WORDS];
    const int64_t c = blockIdx.x;
    const int64_t w0 = c * CHUNK_WORDS;
    const int64_t wn = nwords - w0 < CHUNK_WORDS ? nwords - w0 : CHUNK_WORDS;
#pragma unroll
    for (int u = 0; u < CHUNK_WORDS / BT; ++u) {
        const int64_t q = threadIdx.x + u * BT;
        if (q < wn) words[q] = s_cur[w0 + q];
    }
    const int64_t p0 = off[c * Nb], p1 = off[(c + 1) * Nb];
    const int64_t len = p1 - p0, S = gridDim.y;
    const int64_t a = p0 + len * (int64_t)blockIdx.y / S;
    const int64_t e = p0 + len * ((int64_t)blockIdx.y + 1) / S;
    __syncthreads();
    const int vsh = 6 - shiftG;
    const uint32_t vmask = (1u << vsh) - 1, gmask = (1u << (1 << shiftG)) - 1;
    constexpr int U = 8;
    for (int64_t p = a + threadIdx.x; p < e; p += (int64_t)U * BT) {
        uint32_t r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = p + (int64_t)u * BT;
            r[u] = q < e ? src[q] : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = p + (int64_t)u * BT;
            if (q < e) {
                const uint64_t word = words[r[u] >> vsh];
                bits[q] = (uint8_t)((word >> ((r[u] & vmask) << shiftG)) & gmask);
            }
        }
    }
}

// Pass 2.  One workgroup per bin of B = BIN_WORDS L / G rows; dynamic LDS holds the run
// starts and prefix lengths of the bin's Nc runs (2 (Nc + 1) int32), so that two
// workgroups share a compute unit and one's loads overlap the other's arithmetic.  For
// L > 1 a table in LDS spreads a (flipped) spin byte into the G / L words of its lanes.
template <int L>
__global__ void __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(8))) k_bin_update(
    int64_t n, int shiftG, int64_t Nb, int64_t Nc, int64_t nwords,
    const int32_t *__restrict__ off, const uint8_t *__restrict__ bits,
    const uint32_t *__restrict__ drec, const int32_t *__restrict__ crow,
    uint64_t *__restrict__ s_nxt, float *__restrict__ x, float *__restrict__ m,
    float *__restrict__ h_last, int t, const float *__restrict__ lam, float eta, float alpha) {
    constexpr int LW = 32 / L;                          // lane width in bits
    constexpr uint32_t LMASK = L == 1 ? 0xffffffffu : (1u << LW) - 1;
    constexpr int SUMS = BIN_WORDS * L;                 // (row, replica) sums of a bin
    __shared__ uint32_t acc[BIN_WORDS];
    __shared__ uint32_t spread[L > 1 ? 256 * 8 / L : 1];
    __shared__ int32_t wsum[BT / 64];
    extern __shared__ int32_t runs[];
    int32_t *st = runs;               // start of the run of chunk c
    int32_t *pre = runs + Nc + 1;     // entries of the bin before chunk c's run
    const int64_t bin = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    const int G = 1 << shiftG;
    const int WPE = G / L;            // words of one entry (L <= G)
    const uint32_t gmask = (1u << G) - 1;
    for (int q = tid; q < BIN_WORDS; q += BT) acc[q] = 0u;
    if (L > 1)
        for (int e = tid; e < 256 * WPE; e += BT) {
            const uint32_t byte = (uint32_t)(e / WPE), k = (uint32_t)(e % WPE);
            uint32_t v = 0u;
            for (int l = 0; l < L; ++l) v |= ((byte >> (k * L + l)) & 1u) << (LW * l);
            spread[e] = v;
        }
    // run of chunk c in this bin: [off[c*Nb + bin], off[c*Nb + bin + 1])
    int32_t v[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int64_t c = 2 * tid + u;
        v[u] = 0;
        if (c < Nc) {
            const int32_t a0 = off[c * Nb + bin];
            st[c] = a0;
            v[u] = off[c * Nb + bin + 1] - a0;
        }
    }
    const int32_t total = block_scan_excl<2>(v, wsum);
#pragma unroll
    for (int u = 0; u < 2; ++u)
        if (2 * tid + u < Nc) pre[2 * tid + u] = v[u];
    if (tid == 0) pre[Nc] = total;
    __syncthreads();
    constexpr int U = 8;
    for (int32_t e0 = tid; e0 < total; e0 += U * BT) {
        uint32_t rec[U];
        uint32_t bv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t e = e0 + u * BT;
            rec[u] = 0;
            bv[u] = 0;
            if (e < total) {
                // chunk of entry e: largest c with pre[c] <= e (pre[Nc] = total > e)
                int32_t lo = 0, hi = (int32_t)Nc;
                while (hi - lo > 1) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (pre[mid] <= e) lo = mid;
                    else hi = mid;
                }
                const int64_t p = (int64_t)st[lo] + (e - pre[lo]);
                rec[u] = drec[p];
                bv[u] = bits[p];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (e0 + u * BT >= total) continue;
            const int32_t wv = (int32_t)rec[u] >> 16;
            const uint32_t aw = (uint32_t)(wv < 0 ? -wv : wv);
            const uint32_t fb = bv[u] ^ (wv < 0 ? gmask : 0u);        // b' of each replica
            uint32_t *a = acc + ((rec[u] & 0xffffu) << shiftG) / L;
            if (L == 1) {
                for (int r = 0; r < G; ++r)
                    if ((fb >> r) & 1u) atomicAdd(a + r, aw);
            } else {
                for (int k = 0; k < WPE; ++k) atomicAdd(a + k, aw * spread[fb * WPE + k]);
            }
        }
    }
    __syncthreads();
    // fused update of the bin's (row, replica) pairs; state index = row * G + replica.
    // UQ pairs per thread per round: every load of a round is issued before its stores.
    // x and m stream through once per step (gigabytes, far beyond the caches): their
    // loads and stores are non-temporal, leaving the caches to the entry records.
    constexpr int UQ = 4;
    static_assert((BIN_WORDS / BT) % UQ == 0, "rounds must cover the bin exactly");
    const int64_t q0 = bin * SUMS;
    const float lt = lam[t];
    for (int qb = tid; qb < SUMS; qb += UQ * BT) {
        float xv[UQ], mv[UQ];
        int32_t cr[UQ];
        bool live[UQ];
#pragma unroll
        for (int u = 0; u < UQ; ++u) {
            const int64_t gi = q0 + qb + u * BT;
            live[u] = (gi >> shiftG) < n;
            xv[u] = mv[u] = 0.0f;
            cr[u] = 0;
            if (live[u]) {
                xv[u] = __builtin_nontemporal_load(&x[gi]);
                mv[u] = __builtin_nontemporal_load(&m[gi]);
                cr[u] = crow[gi >> shiftG];
            }
        }
#pragma unroll
        for (int u = 0; u < UQ; ++u) {
            const int q = qb + u * BT;
            const int64_t gi = q0 + q;
            bool neg = false;
            if (live[u]) {
                const int32_t A = (int32_t)((acc[q / L] >> (LW * (q % L))) & LMASK);
                const float h = (float)(cr[u] - 2 * A);
                pa_update(h, lt, eta, alpha, xv[u], mv[u]);
                __builtin_nontemporal_store(xv[u], &x[gi]);
                __builtin_nontemporal_store(mv[u], &m[gi]);
                if (h_last) h_last[gi] = h;
                neg = xv[u] < 0.0f;
            }
            const uint64_t bal = __ballot(neg);
            const int64_t wi = (gi - lane) >> 6;
            if (lane == 0 && wi < nwords) s_nxt[wi] = bal;
        }
    }
}

int ilog2(int64_t v) {
    int s = 0;
    while (((int64_t)1 << s) < v) ++s;
    return s;
}

}  // namespace

bool bin_geometry(int64_t n, int G, int lanes, BinGeom &g) {
    if (G < 1 || G > 8 || (G & (G - 1)) != 0 || n < 1) return false;
    if (lanes != 1 && lanes != 2 && lanes != 4) return false;
    if (lanes > G) return false;
    g.G = G;
    g.lanes = lanes;
    g.shiftG = ilog2(G);
    g.cshift = 20 - g.shiftG;                    // C * G / 64 = CHUNK_WORDS
    g.bshift = 14 + ilog2(lanes) - g.shiftG;     // B * G = BIN_WORDS * lanes
    g.Nc = (n + ((int64_t)1 << g.cshift) - 1) >> g.cshift;
    g.Nb = (n + ((int64_t)1 << g.bshift) - 1) >> g.bshift;
    g.M = g.Nc * g.Nb;
    return g.Nc <= BIN_MAX_CHUNKS && g.M < ((int64_t)1 << 31) - SCAN_TILE;
}

int64_t bin_scan_tiles(const BinGeom &g) { return (g.M + SCAN_TILE - 1) / SCAN_TILE; }

hipError_t launch_bin_build(const CsrView &c, const BinGeom &g, const int64_t *b_i64,
                            int32_t *off, int32_t *cur, int32_t *tsum, uint32_t *src,
                            uint32_t *drec, int32_t *crow, hipStream_t st) {
    const unsigned rows = (unsigned)((c.n + 255) / 256);
    int64_t fg = (g.M + 255) / 256;
    if (fg > 65536) fg = 65536;
    k_bin_fill<<<(unsigned)fg, 256, 0, st>>>(cur, g.M);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    auto byi = [&](auto itag) -> hipError_t {
        using TI = decltype(itag);
        const TI *col = static_cast<const TI *>(c.col);
        k_bin_count<TI><<<rows, 256, 0, st>>>(c.n, c.rp, col, c.skip_diag, g.cshift, g.bshift,
                                              g.Nb, cur);
        hipError_t e2 = hipGetLastError();
        if (e2 != hipSuccess) return e2;
        const int64_t nt = bin_scan_tiles(g);
        k_bin_tile_sums<<<(unsigned)nt, BT, 0, st>>>(cur, g.M, tsum);
        k_bin_scan_tiles<<<1, BT, 0, st>>>(tsum, nt, off, g.M);
        k_bin_offsets<<<(unsigned)nt, BT, 0, st>>>(cur, g.M, tsum, off, cur);
        e2 = hipGetLastError();
        if (e2 != hipSuccess) return e2;
        if (c.w_dt == QPA_I8) {
            const int8_t *w = static_cast<const int8_t *>(c.w);
            k_bin_scatter<TI, int8_t><<<rows, 256, 0, st>>>(c.n, c.rp, col, w, c.skip_diag,
                                                            g.cshift, g.bshift, g.Nb, cur, src,
                                                            drec);
            k_bin_rowconst<TI, int8_t><<<rows, 256, 0, st>>>(c.n, c.rp, col, w, c.skip_diag,
                                                             b_i64, crow);
        } else {
            const int16_t *w = static_cast<const int16_t *>(c.w);
            k_bin_scatter<TI, int16_t><<<rows, 256, 0, st>>>(c.n, c.rp, col, w, c.skip_diag,
                                                             g.cshift, g.bshift, g.Nb, cur, src,
                                                             drec);
            k_bin_rowconst<TI, int16_t><<<rows, 256, 0, st>>>(c.n, c.rp, col, w, c.skip_diag,
                                                              b_i64, crow);
        }
        return hipGetLastError();
    };
    if (c.w_dt != QPA_I8 && c.w_dt != QPA_I16) return hipErrorInvalidValue;
    return c.col_dt == QPA_I16 ? byi((int16_t)0) : byi((int32_t)0);
}

hipError_t launch_bin_step(const BinGeom &g, int64_t n, int64_t nwords, const int32_t *off,
                           const uint32_t *src, const uint32_t *drec, uint8_t *bits,
                           const int32_t *crow, const uint64_t *s_cur, uint64_t *s_nxt, float *x,
                           float *m, float *h_last, int32_t t, const float *lam, float eta,
                           float alpha, int cus, hipStream_t st) {
    int64_t S = (4 * (int64_t)cus + g.Nc - 1) / g.Nc;
    if (S < 1) S = 1;
    if (S > 64) S = 64;
    k_bin_gather<<<dim3((unsigned)g.Nc, (unsigned)S), BT, 0, st>>>(g.shiftG, nwords, g.Nb, off,
                                                                   src, s_cur, bits);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds = sizeof(int32_t) * 2 * (size_t)(g.Nc + 1);
    const unsigned nb = (unsigned)g.Nb;
    if (g.lanes == 4)
        k_bin_update<4><<<nb, BT, lds, st>>>(n, g.shiftG, g.Nb, g.Nc, nwords, off, bits, drec,
                                             crow, s_nxt, x, m, h_last, t, lam, eta, alpha);
    else if (g.lanes == 2)
        k_bin_update<2><<<nb, BT, lds, st>>>(n, g.shiftG, g.Nb, g.Nc, nwords, off, bits, drec,
                                             crow, s_nxt, x, m, h_last, t, lam, eta, alpha);
    else
        k_bin_update<1><<<nb, BT, lds, st>>>(n, g.shiftG, g.Nb, g.Nc, nwords, off, bits, drec,
                                             crow, s_nxt, x, m, h_last, t, lam, eta, alpha);
    return hipGetLastError();
}

}  // namespace qpa
