// Dense PA steps in FP32 (App. B).  Every kernel accumulates each local field
// sum_j J_ij s_j in ascending j from zero and then adds b_i: with s = +-1 every product is
// exact, so the result is the same FP32 sum whatever the tiling, and trajectories are
// reproducible bit for bit.  For the same reason a fused multiply-add s_j J_ij + acc,
// rounded once, equals the separately rounded product and sum, in one instruction.
//
// The update after the field is, each operation rounded separately:
//   g = lambda_t * x + h;  m' = alpha * m - eta * g;  x' = clip(x + m', -1, 1).
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

__device__ __forceinline__ float spin_of(float x) { return x >= 0.0f ? 1.0f : -1.0f; }

// ---------------------------------------------------------------- LDS-resident (small n)
// A block owns RB replicas and all n variables for every step in [t0, t1): couplings,
// fields and both spin buffers live in LDS, analog state in registers.  Thread p of the
// block handles pairs p, p + 256, ... of the RB x n (replica, variable) grid.
constexpr int RES_THREADS = 256;
constexpr int RES_PAIRS = 2;

__global__ void __launch_bounds__(RES_THREADS) k_dense_resident(
    int n, int R, int RB, const float *__restrict__ J, const float *__restrict__ b,
    float *__restrict__ x, float *__restrict__ m, float *__restrict__ h_last, int t0, int t1,
    const float *__restrict__ lam, float eta, float alpha) {
    extern __shared__ float sh[];
    float *sJ = sh;
    float *sb = sJ + n * n;
    float *sS = sb + n;   // [2][RB][n]
    const int tid = threadIdx.x;
    const int r0 = blockIdx.x * RB;
    const int nr = min(RB, R - r0);
    for (int k = tid; k < n * n; k += RES_THREADS) sJ[k] = J[k];
    for (int k = tid; k < n; k += RES_THREADS) sb[k] = b[k];

    float xr[RES_PAIRS], mr[RES_PAIRS], hr[RES_PAIRS];
    int rl[RES_PAIRS], iv[RES_PAIRS];
    bool act[RES_PAIRS];
#pragma unroll
    for (int q = 0; q < RES_PAIRS; ++q) {
        int p = tid + q * RES_THREADS;
        act[q] = p < nr * n;
        rl[q] = act[q] ? p / n : 0;
        iv[q] = act[q] ? p - rl[q] * n : 0;
        xr[q] = mr[q] = hr[q] = 0.0f;
        if (act[q]) {
            int64_t g = (int64_t)(r0 + rl[q]) * n + iv[q];
            xr[q] = x[g];
            mr[q] = m[g];
            sS[rl[q] * n + iv[q]] = spin_of(xr[q]);
        }
    }
    __syncthreads();
    int cur = 0;
    for (int t = t0; t < t1; ++t) {
        const float lt = lam[t];
        const float *scur = sS + cur * RB * n;
        float *snxt = sS + (cur ^ 1) * RB * n;
#pragma unroll
        for (int q = 0; q < RES_PAIRS; ++q) {
            if (!act[q]) continue;
            const float *Jrow = sJ + iv[q] * n;
            const float *srow = scur + rl[q] * n;
            float acc = 0.0f;
            for (int j = 0; j < n; ++j) acc = __fmaf_rn(Jrow[j], srow[j], acc);
            float h = __fadd_rn(acc, sb[iv[q]]);
            hr[q] = h;
            pa_update(h, lt, eta, alpha, xr[q], mr[q]);
            snxt[rl[q] * n + iv[q]] = spin_of(xr[q]);
        }
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int q = 0; q < RES_PAIRS; ++q) {
        if (!act[q]) continue;
        int64_t g = (int64_t)(r0 + rl[q]) * n + iv[q];
        x[g] = xr[q];
        m[g] = mr[q];
        if (h_last && t1 > t0) h_last[g] = hr[q];
    }
}

// ---------------------------------------------------------------- one wave per replica
// n <= 64: lane i holds row i of J (NW >= n registers), x_i and m_i.  The spins of a step
// are one 64-bit ballot (bit j set <=> x_j < 0), so the sign of term j is the same in every
// lane, and J_ij * s_j is J_ij with its sign bit flipped where s_j = -1 (the FP32 product,
// exactly).  The sums ascend in j from zero as in the block kernel; no LDS, no barrier.
// The schedule is read 64 steps at a time, one value per lane.
template <int NW>
__global__ void __launch_bounds__(64) k_dense_wave(int n, const float *__restrict__ J,
                                                   const float *__restrict__ b,
                                                   float *__restrict__ x, float *__restrict__ m,
                                                   float *__restrict__ h_last, int t0, int t1,
                                                   const float *__restrict__ lam, float eta,
                                                   float alpha) {
    const int i = threadIdx.x;
    const bool act = i < n;
    const int64_t g = (int64_t)blockIdx.x * n + i;
    float Jr[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) Jr[j] = (act && j < n) ? J[(int64_t)i * n + j] : 0.0f;
    float xi = 0.0f, mi = 0.0f, bi = 0.0f, hi = 0.0f;
    if (act) {
        xi = x[g];
        mi = m[g];
        bi = b[i];
    }
    uint64_t neg = __ballot(act && xi < 0.0f);
    for (int tb = t0; tb < t1; tb += 64) {
        const float lv = tb + i < t1 ? lam[tb + i] : 0.0f;
        const int te = t1 - tb < 64 ? t1 - tb : 64;
        for (int k = 0; k < te; ++k) {
            const float lt = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lv), k));
            float acc = 0.0f;
            // terms j >= n are +0.0 (zero coupling, spin bit clear): a sum that starts at
            // +0.0 never becomes -0.0 under round-to-nearest, so adding them changes no bit
#pragma unroll
            for (int j = 0; j < NW; ++j) {
                const uint32_t sgn = (uint32_t)((neg >> j) & 1u) << 31;
                acc = __fadd_rn(acc, __uint_as_float(__float_as_uint(Jr[j]) ^ sgn));
            }
            hi = __fadd_rn(acc, bi);
            pa_update(hi, lt, eta, alpha, xi, mi);
            neg = __ballot(act && xi < 0.0f);
        }
    }
    if (act) {
        x[g] = xi;
        m[g] = mi;
        if (h_last && t1 > t0) h_last[g] = hi;
    }
}


__global__ void __launch_bounds__(256) k_sign_f32(int64_t count, const float *__restrict__ x,
                                                  float *__restrict__ s) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * blockDim.x)
        s[k] = spin_of(x[k]);
}

int resident_rb(int64_t n) {
    int rb = (int)((RES_THREADS * RES_PAIRS) / n);
    return rb < 1 ? 1 : rb;
}

size_t resident_lds_bytes(int64_t n) {
    return sizeof(float) * (size_t)(n * n + n + 2 * resident_rb(n) * n);
}

}  // namespace

bool dense_resident_fits(int64_t n) {
    return n >= 1 && n <= 128 && resident_lds_bytes(n) <= 64 * 1024;
}

hipError_t launch_dense_resident(int64_t n, int64_t R, const float *J, const float *b,
                                 float *x, float *m, float *h_last, int32_t t0, int32_t t1,
                                 const float *lam, float eta, float alpha, hipStream_t st) {
    if (!dense_resident_fits(n)) return hipErrorInvalidValue;
    if (n <= 64 && R <= INT32_MAX) {
        const unsigned grid = (unsigned)R;
        if (n <= 16)
            k_dense_wave<16><<<grid, 64, 0, st>>>((int)n, J, b, x, m, h_last, t0, t1, lam, eta,
                                                  alpha);
        else if (n <= 32)
            k_dense_wave<32><<<grid, 64, 0, st>>>((int)n, J, b, x, m, h_last, t0, t1, lam, eta,
                                                  alpha);
        else
            k_dense_wave<64><<<grid, 64, 0, st>>>((int)n, J, b, x, m, h_last, t0, t1, lam, eta,
                                                  alpha);
        return hipGetLastError();
    }
    const int rb = resident_rb(n);
    const unsigned grid = (unsigned)((R + rb - 1) / rb);
    const size_t lds = resident_lds_bytes(n);
    k_dense_resident<<<grid, RES_THREADS, lds, st>>>((int)n, (int)R, rb, J, b, x, m, h_last,
                                                     t0, t1, lam, eta, alpha);
    return hipGetLastError();
}

hipError_t launch_sign_f32(int64_t count, const float *x, float *s, hipStream_t st) {
    if (count == 0) return hipSuccess;
    int64_t g = (count + 255) / 256;
    if (g > 65536) g = 65536;
    k_sign_f32<<<(unsigned)g, 256, 0, st>>>(count, x, s);
    return hipGetLastError();
}

}  // namespace qpa
