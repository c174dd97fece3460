// Batched PA (App. B) over many uneven sparse instances in one persistent launch.
//
// A task is (instance, group of up to 64 replicas).  Tasks are listed largest first
// (by stored entries) and handed out through an atomic counter: every workgroup keeps
// taking the next task until the list is exhausted, so each workgroup runs whole tasks
// and no two workgroups ever wait on each other.  Inside a task the workgroup owns all
// variables of its replicas for all steps:
//   * lane = replica (64 lanes per wave), so one CSR entry serves 64 replicas at once;
//   * the spins of variable j for the 64 replicas are one 64-bit word in LDS (bit set
//     <=> spin -1), double buffered across the synchronous step;
//   * a row's entries are fetched 64 at a time by the wave's lanes and then walked one by
//     one with lane broadcasts, so a coupling is read from memory once per step;
//   * analog state x, m lives in the task's slice of the workspace, [n][64] FP32
//     (replica fastest, 256 contiguous bytes per variable).
// Field sums follow the definition's entry order (int32 exact for integer couplings,
// FP32 in row order for float couplings); the update is the same FP32 sequence as the
// single-instance kernels.  The initial state of replica r (global index within its
// instance) is drawn from SplitMix64 output number r*n + i + 1 of the instance's seed.
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

__device__ __forceinline__ uint64_t splitmix_output(uint64_t seed, uint64_t k) {
    uint64_t z = seed + k * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

template <typename T> __device__ __forceinline__ T ldv(const void *p, int64_t k) {
    return static_cast<const T *>(p)[k];
}

// Weight k of a row as int32 / float, index k as int64, for the caller's dtypes.
__device__ __forceinline__ int32_t weight_i(const BatchTask &tk, int64_t k) {
    switch (tk.w_dt) {
        case QPA_I8: return ldv<int8_t>(tk.w, k);
        case QPA_I16: return ldv<int16_t>(tk.w, k);
        default: return ldv<int32_t>(tk.w, k);
    }
}
__device__ __forceinline__ float weight_f(const BatchTask &tk, int64_t k) {
    switch (tk.w_dt) {
        case QPA_I8: return (float)ldv<int8_t>(tk.w, k);
        case QPA_I16: return (float)ldv<int16_t>(tk.w, k);
        case QPA_I32: return (float)ldv<int32_t>(tk.w, k);
        default: return ldv<float>(tk.w, k);
    }
}
__device__ __forceinline__ int64_t column(const BatchTask &tk, int64_t k) {
    return tk.col_dt == QPA_I16 ? (int64_t)ldv<int16_t>(tk.col, k) : (int64_t)ldv<int32_t>(tk.col, k);
}

constexpr int BT_THREADS = 256;
constexpr int BT_WAVES = BT_THREADS / 64;

__global__ void __launch_bounds__(BT_THREADS) k_csr_batch(const BatchTask *__restrict__ tasks,
                                                          int32_t ntasks,
                                                          int32_t *__restrict__ next_task,
                                                          int32_t T, const float *__restrict__ lam,
                                                          float eta, float alpha, float sigma0,
                                                          int32_t max_n) {
    extern __shared__ uint64_t spins[];        // [2][max_n]
    __shared__ int32_t cur_task;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    for (;;) {
        if (threadIdx.x == 0) cur_task = atomicAdd(next_task, 1);
        __syncthreads();
        const int32_t task = cur_task;
        __syncthreads();
        if (task >= ntasks) break;             // every wave of the workgroup leaves together
        const BatchTask tk = tasks[task];
        const int64_t n = tk.n;
        const int64_t r = (int64_t)tk.group * 64 + lane;   // replica index in the instance
        const bool live = lane < tk.nrep;
        float *xs = tk.x, *ms = tk.m;
        uint64_t *s0 = spins, *s1 = spins + max_n;

        // initial state and spins
        for (int64_t i = wv; i < n; i += BT_WAVES) {
            float xv = 0.0f;
            if (live) {
                uint64_t top = splitmix_output(tk.seed, (uint64_t)(r * n + i) + 1u) >> 40;
                float u = __fmul_rn((float)top, 1.0f / 16777216.0f);
                float v = __fsub_rn(__fmul_rn(2.0f, u), 1.0f);
                xv = __fmul_rn(sigma0, v);
            }
            xs[i * 64 + lane] = xv;
            ms[i * 64 + lane] = 0.0f;
            uint64_t bal = __ballot(xv < 0.0f);
            if (lane == 0) s0[i] = bal;
        }
        __syncthreads();

        for (int32_t t = 0; t < T; ++t) {
            const float lt = lam[t];
            for (int64_t i = wv; i < n; i += BT_WAVES) {
                const int64_t k0 = tk.rp[i], k1 = tk.rp[i + 1];
                int32_t ai = 0;
                float af = 0.0f;
                for (int64_t kb = k0; kb < k1; kb += 64) {
                    // lanes fetch up to 64 entries, then the wave walks them in order
                    const int64_t kk = kb + lane;
                    int64_t cj = -1;
                    int32_t wi = 0;
                    float wf = 0.0f;
                    if (kk < k1) {
                        cj = column(tk, kk);
                        if (tk.is_int) wi = weight_i(tk, kk);
                        else wf = weight_f(tk, kk);
                    }
                    const int cnt = (int)min((int64_t)64, k1 - kb);
                    for (int e = 0; e < cnt; ++e) {
                        const int64_t j = __shfl(cj, e);
                        if (tk.skip_diag && j == i) continue;
                        const uint64_t word = s0[j];
                        const bool neg = (word >> lane) & 1u;
                        if (tk.is_int) {
                            const int32_t we = __shfl(wi, e);
                            ai += neg ? -we : we;
                        } else {
                            const float we = __shfl(wf, e);
                            af = __fadd_rn(af, neg ? -we : we);
                        }
                    }
                }
                const float bi = tk.b[i];
                const float h = tk.is_int ? __fadd_rn((float)ai, bi) : __fadd_rn(af, bi);
                float xv = xs[i * 64 + lane], mv = ms[i * 64 + lane];
                pa_update(h, lt, eta, alpha, xv, mv);
                xs[i * 64 + lane] = xv;
                ms[i * 64 + lane] = mv;
                const uint64_t bal = __ballot(xv < 0.0f);
                if (lane == 0) s1[i] = bal;
            }
            __syncthreads();
            uint64_t *tmp = s0;
            s0 = s1;
            s1 = tmp;
        }
        __syncthreads();
    }
}

}  // namespace

size_t batch_lds_bytes(int32_t max_n) { return sizeof(uint64_t) * 2 * (size_t)max_n; }

hipError_t launch_csr_batch(const BatchTask *tasks, int32_t ntasks, int32_t *next_task,
                            int32_t blocks, int32_t T, const float *lam, float eta, float alpha,
                            float sigma0, int32_t max_n, hipStream_t st) {
    const size_t lds = batch_lds_bytes(max_n);
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    hipError_t e = hipMemsetAsync(next_task, 0, sizeof(int32_t), st);
    if (e != hipSuccess) return e;
    k_csr_batch<<<blocks, BT_THREADS, lds, st>>>(tasks, ntasks, next_task, T, lam, eta, alpha,
                                                 sigma0, max_n);
    return hipGetLastError();
}

}  // namespace qpa
