// Low-energy spectrum of a sample set (the many low-energy states a run returns,
// Sec. V.A): the distinct states among R replicas, ordered by energy and then by the
// lowest replica index holding them, with their multiplicities.
//
// 1. k_spec_pack: one wave per replica packs its int8 spins into 64-bit words (one
//    ballot per 64 variables, bit set <=> spin -1) and folds the words into a 64-bit
//    hash (sum over words of a SplitMix64-style finaliser of word + position).
// 2. k_spec_select: one workgroup sorts (energy, hash, replica) with a bitonic network
//    in LDS; equal (energy, hash) runs are groups.  A group whose members all equal its
//    first member (compared word by word) is one state: its first member represents it
//    and its size is the count.  A group holding distinct states (a hash collision) is
//    resolved by pairwise comparison.  The representatives are then sorted by
//    (energy, replica) and the first k written out.
// 3. k_spec_gather: copies the spins of the selected replicas.
#include "qpa_internal.h"

namespace qpa {
namespace {

constexpr int SPEC_THREADS = 1024;

__device__ __forceinline__ uint64_t spec_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256) k_spec_pack(int64_t n, int32_t R, int64_t nw,
                                                   const int8_t *__restrict__ spins,
                                                   int32_t no_hash,
                                                   uint64_t *__restrict__ bits,
                                                   uint64_t *__restrict__ hash) {
    const int lane = threadIdx.x & 63;
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (r >= R) return;
    const int8_t *s = spins + r * n;
    uint64_t h = 0;
    for (int64_t w = 0; w < nw; ++w) {
        const int64_t i = 64 * w + lane;
        const bool neg = i < n && s[i] < 0;
        const uint64_t word = __ballot(neg);
        if (lane == 0) bits[r * nw + w] = word;
        h += spec_mix(word + (uint64_t)(w + 1) * 0x9e3779b97f4a7c15ull);
    }
    if (lane == 0) hash[r] = no_hash ? 0ull : h;
}

__device__ __forceinline__ bool spec_equal(const uint64_t *__restrict__ bits, int64_t nw,
                                           int32_t a, int32_t b) {
    if (a == b) return true;
    const uint64_t *x = bits + (int64_t)a * nw, *y = bits + (int64_t)b * nw;
    for (int64_t w = 0; w < nw; ++w)
        if (x[w] != y[w]) return false;
    return true;
}

// order-preserving unsigned key of a double (-0 is folded into +0 first)
__device__ __forceinline__ uint64_t spec_ekey(double e) {
    const uint64_t u = (uint64_t)__double_as_longlong(e + 0.0);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// Bitonic sort of RP (a power of two) entries by (ka, kb) ascending.  Live entries carry
// distinct (ka, kb) pairs, so their order is unique; padding sorts last.
__device__ void spec_sort(int32_t RP, uint64_t *ka, uint64_t *kb) {
    for (int32_t size = 2; size <= RP; size <<= 1) {
        for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int32_t i = threadIdx.x; i < RP; i += SPEC_THREADS) {
                const int32_t j = i ^ stride;
                if (j <= i) continue;
                const bool up = (i & size) == 0;
                const bool gt = ka[i] > ka[j] || (ka[i] == ka[j] && kb[i] > kb[j]);
                if (gt == up) {
                    uint64_t x = ka[i];
                    ka[i] = ka[j];
                    ka[j] = x;
                    x = kb[i];
                    kb[i] = kb[j];
                    kb[j] = x;
                }
            }
            __syncthreads();
        }
    }
}

constexpr int SPEC_IBITS = 12;                       // replica index bits in a sort key
constexpr uint64_t SPEC_IMASK = (1ull << SPEC_IBITS) - 1;

// LDS: ek, kb (u64) and gs, gc, cnt (i32), RP entries each.  First sort key: the
// energy, then the hash (top 52 bits) with the replica index in the low 12 bits, so
// that equal (energy, hash) runs are ordered by replica.
__global__ void __launch_bounds__(SPEC_THREADS) k_spec_select(
    int32_t R, int32_t RP, int64_t nw, const double *__restrict__ energy,
    const uint64_t *__restrict__ bits, const uint64_t *__restrict__ hash, int32_t k,
    double *__restrict__ out_energy, int32_t *__restrict__ out_count,
    int32_t *__restrict__ out_first, int32_t *__restrict__ out_distinct) {
    extern __shared__ uint64_t spec_lds[];
    uint64_t *ek = spec_lds;
    uint64_t *kb = ek + RP;
    int32_t *gs = reinterpret_cast<int32_t *>(kb + RP);   // group start of a position
    int32_t *gc = gs + RP;     // at a group start: group size; bit 31: mixed group
    int32_t *cnt = gc + RP;    // count of a representative, 0 otherwise
    __shared__ int32_t ndist;
    const int32_t t = threadIdx.x;
    for (int32_t i = t; i < RP; i += SPEC_THREADS) {
        if (i < R) {
            ek[i] = spec_ekey(energy[i]);
            kb[i] = (hash[i] << SPEC_IBITS) | (uint64_t)i;
        } else {
            ek[i] = ~0ull;
            kb[i] = ~0ull;
        }
        gc[i] = 0;
        cnt[i] = 0;
    }
    if (t == 0) ndist = 0;
    __syncthreads();
    spec_sort(RP, ek, kb);
    for (int32_t i = t; i < R; i += SPEC_THREADS) {
        const bool head = i == 0 || ek[i] != ek[i - 1] ||
                          (kb[i] >> SPEC_IBITS) != (kb[i - 1] >> SPEC_IBITS);
        gs[i] = head ? i : 0;
    }
    __syncthreads();
    // group start = largest head position <= i (prefix max; R <= 4 * SPEC_THREADS)
    for (int32_t off = 1; off < R; off <<= 1) {
        int32_t v[4];
        int c = 0;
        for (int32_t i = t; i < R; i += SPEC_THREADS, ++c)
            v[c] = (i >= off && gs[i - off] > gs[i]) ? gs[i - off] : gs[i];
        __syncthreads();
        c = 0;
        for (int32_t i = t; i < R; i += SPEC_THREADS, ++c) gs[i] = v[c];
        __syncthreads();
    }
    for (int32_t i = t; i < R; i += SPEC_THREADS) atomicAdd(&gc[gs[i]], 1);
    __syncthreads();
    // groups whose members are not all equal to the first one (hash collisions)
    for (int32_t i = t; i < R; i += SPEC_THREADS) {
        const int32_t g0 = gs[i];
        if (!spec_equal(bits, nw, (int32_t)(kb[i] & SPEC_IMASK), (int32_t)(kb[g0] & SPEC_IMASK)))
            atomicOr(&gc[g0], (int32_t)0x80000000);
    }
    __syncthreads();
    for (int32_t i = t; i < R; i += SPEC_THREADS) {
        const int32_t g0 = gs[i];
        const int32_t gsz = gc[g0] & 0x7fffffff;
        const int32_t ri = (int32_t)(kb[i] & SPEC_IMASK);
        int32_t c = 0;
        if (!(gc[g0] & (int32_t)0x80000000)) {
            c = (i == g0) ? gsz : 0;
        } else {
            // first position of its state inside the group (the group is in replica
            // order), then the number of members equal to it
            bool first = true;
            for (int32_t j = g0; j < i && first; ++j)
                if (spec_equal(bits, nw, ri, (int32_t)(kb[j] & SPEC_IMASK))) first = false;
            if (first)
                for (int32_t j = g0; j < g0 + gsz; ++j)
                    c += spec_equal(bits, nw, ri, (int32_t)(kb[j] & SPEC_IMASK));
        }
        cnt[i] = c;
        if (c) atomicAdd(&ndist, 1);
    }
    __syncthreads();
    // representatives by (energy, replica); the count rides in the low half of the key
    for (int32_t i = t; i < RP; i += SPEC_THREADS) {
        if (i < R && cnt[i]) {
            kb[i] = ((kb[i] & SPEC_IMASK) << 32) | (uint32_t)cnt[i];
        } else {
            ek[i] = ~0ull;
            kb[i] = ~0ull;
        }
    }
    __syncthreads();
    spec_sort(RP, ek, kb);
    const int32_t m = ndist < k ? ndist : k;
    for (int32_t i = t; i < m; i += SPEC_THREADS) {
        const int32_t r = (int32_t)(kb[i] >> 32);
        out_first[i] = r;
        out_count[i] = (int32_t)(kb[i] & 0xffffffffu);
        out_energy[i] = energy[r];
    }
    if (t == 0) out_distinct[0] = ndist;
}

__global__ void __launch_bounds__(256) k_spec_gather(int64_t n, int32_t k,
                                                     const int8_t *__restrict__ spins,
                                                     const int32_t *__restrict__ first,
                                                     const int32_t *__restrict__ ndist,
                                                     int8_t *__restrict__ out) {
    const int32_t m = ndist[0] < k ? ndist[0] : k;
    const int64_t total = (int64_t)m * n;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = q / n, i = q - row * n;
        out[q] = spins[(int64_t)first[row] * n + i];
    }
}

}  // namespace

size_t spectrum_lds_bytes(int32_t RP) { return (size_t)RP * 28; }

hipError_t launch_spectrum(int64_t n, int32_t R, const int8_t *spins, const double *energy,
                           int32_t k, int32_t no_hash, uint64_t *bits, uint64_t *hash,
                           int8_t *out_spins, double *out_energy, int32_t *out_count,
                           int32_t *out_first, int32_t *out_distinct, hipStream_t st) {
    const int64_t nw = (n + 63) / 64;
    k_spec_pack<<<(unsigned)((R + 3) / 4), 256, 0, st>>>(n, R, nw, spins, no_hash, bits, hash);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int32_t RP = 1;
    while (RP < R) RP <<= 1;
    const size_t lds = spectrum_lds_bytes(RP);
    if (lds > 64 * 1024) {
        e = hipFuncSetAttribute((const void *)k_spec_select,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    k_spec_select<<<1, SPEC_THREADS, lds, st>>>(R, RP, nw, energy, bits, hash, k, out_energy,
                                                out_count, out_first, out_distinct);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (out_spins && k > 0) {
        const int64_t total = (int64_t)(k < R ? k : R) * n;
        int64_t g = (total + 255) / 256;
        if (g > 65536) g = 65536;
        k_spec_gather<<<(unsigned)(g < 1 ? 1 : g), 256, 0, st>>>(n, k, spins, out_first,
                                                                 out_distinct, out_spins);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace qpa
