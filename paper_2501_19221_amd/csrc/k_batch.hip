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

constexpr int BT_THREADS = 1024;
constexpr int BT_WAVES = BT_THREADS / 64;

// All steps of one task, for its weight type TW and index type TI (integer instances:
// exact int32 sums; otherwise FP32 sums of +-w in row order, the weight as float).  Wave w takes rows w,
// w + BT_WAVES, ...; a row's entries are fetched 64 at a time by the lanes and broadcast
// one by one (uniform reads), each reading the neighbour's 64 spins as one 64-bit word
// from LDS.
template <typename TW, typename TI>
__device__ __forceinline__ void run_task(const BatchTask &tk, uint64_t *spins, int32_t max_n,
                                         int32_t T, const float *__restrict__ lam, float eta,
                                         float alpha, float sigma0, int lane, int wv) {
    typedef const __attribute__((address_space(1))) TW *gw_t;
    typedef const __attribute__((address_space(1))) TI *gi_t;
    typedef const __attribute__((address_space(1))) int32_t *gr_t;
    const gw_t w = (gw_t)tk.w;
    const gi_t col = (gi_t)tk.col;
    const gr_t rp = (gr_t)tk.rp;
    const int64_t n = tk.n;
    const int64_t r = (int64_t)tk.group * 64 + lane;   // replica index in the instance
    const bool live = lane < tk.nrep;
    const bool skip = tk.skip_diag != 0;
    const bool INT = tk.is_int != 0;
    float *xs = tk.x, *ms = tk.m;
    uint64_t *s0 = spins, *s1 = spins + max_n;
    // this lane's spin is bit (lane % 32) of the low or high half of a variable's word
    const uint32_t sh = (uint32_t)lane & 31u;
    const bool hi = lane >= 32;

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
            // the row's state first: in flight during the walk
            float xv = xs[i * 64 + lane], mv = ms[i * 64 + lane];
            const int32_t k0 = rp[i], k1 = rp[i + 1];
            int32_t ai = 0;
            float af = 0.0f;
            // lanes fetch the row's entries 64 at a time (past the row's end: its last one
            // again, unused), the next window while this one is walked
            auto fetch = [&](int32_t kb, int32_t &cj, int32_t &wq) {
                const int32_t kk = min(kb + lane, max(k1 - 1, k0));
                cj = (int32_t)col[kk];
                const TW wl = w[kk];
                wq = INT ? (int32_t)wl : __float_as_int((float)wl);
            };
            int32_t cj = 0, wq = 0, cjn = 0, wqn = 0;
            if (k1 > k0) fetch(k0, cj, wq);
            for (int32_t kb = k0; kb < k1; kb += 64) {
                fetch(kb + 64, cjn, wqn);
                const int cnt = min(64, k1 - kb);
                // four entries at a time, their spin words read together; slots past the
                // row's end and a stored QUBO diagonal (folded into b) add zero, which is
                // exact: an integer sum, or a float sum that starts at +0 and so is never -0
                for (int e = 0; e < cnt; e += 4) {
                    int32_t j[4], wb[4];
                    uint64_t word[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int ek = min(e + k, cnt - 1);
                        j[k] = __builtin_amdgcn_readlane(cj, ek);
                        const int32_t wr = __builtin_amdgcn_readlane(wq, ek);
                        wb[k] = (e + k < cnt && !(skip && (int64_t)j[k] == i)) ? wr : 0;
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k) word[k] = s0[j[k]];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint32_t half = hi ? (uint32_t)(word[k] >> 32) : (uint32_t)word[k];
                        const bool neg = (half >> sh) & 1u;
                        if (INT) {
                            ai += neg ? -wb[k] : wb[k];
                        } else {
                            const float we = __int_as_float(wb[k]);
                            af = __fadd_rn(af, neg ? -we : we);
                        }
                    }
                }
                cj = cjn;
                wq = wqn;
            }
            const float bi = tk.b[i];
            const float h = INT ? __fadd_rn((float)ai, bi) : __fadd_rn(af, bi);
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

__global__ void __launch_bounds__(BT_THREADS) k_csr_batch(const BatchTask *__restrict__ tasks,
                                                          int32_t ntasks,
                                                          int32_t *__restrict__ next_task,
                                                          int32_t T, const float *__restrict__ lam,
                                                          float eta, float alpha, float sigma0,
                                                          int32_t max_n) {
    extern __shared__ uint64_t spins[];        // [2][max_n]
    __shared__ int32_t cur_task;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (;;) {
        if (threadIdx.x == 0) cur_task = atomicAdd(next_task, 1);
        __syncthreads();
        const int32_t task = cur_task;
        __syncthreads();
        if (task >= ntasks) break;             // every wave of the workgroup leaves together
        const BatchTask tk = tasks[task];
        // one dispatch per task on the caller's dtypes (weights, indices)
        const bool i16 = tk.col_dt == QPA_I16;
#define QPA_TASK(TW, TI) \
    run_task<TW, TI>(tk, spins, max_n, T, lam, eta, alpha, sigma0, lane, wv)
        switch (tk.w_dt) {
            case QPA_I8:
                if (i16) QPA_TASK(int8_t, int16_t); else QPA_TASK(int8_t, int32_t);
                break;
            case QPA_I16:
                if (i16) QPA_TASK(int16_t, int16_t); else QPA_TASK(int16_t, int32_t);
                break;
            case QPA_I32:
                if (i16) QPA_TASK(int32_t, int16_t); else QPA_TASK(int32_t, int32_t);
                break;
            default:
                if (i16) QPA_TASK(float, int16_t); else QPA_TASK(float, int32_t);
                break;
        }
#undef QPA_TASK
    }
}

__global__ void k_zero_counter(int32_t *c) { *c = 0; }

}  // namespace

size_t batch_lds_bytes(int32_t max_n) { return sizeof(uint64_t) * 2 * (size_t)max_n; }

hipError_t launch_csr_batch(const BatchTask *tasks, int32_t ntasks, int32_t *next_task,
                            int32_t blocks, int32_t T, const float *lam, float eta, float alpha,
                            float sigma0, int32_t max_n, hipStream_t st) {
    const size_t lds = batch_lds_bytes(max_n);
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    // the task counter starts at zero (a kernel, not a memset: the launch may be captured)
    k_zero_counter<<<1, 1, 0, st>>>(next_task);
    k_csr_batch<<<blocks, BT_THREADS, lds, st>>>(tasks, ntasks, next_task, T, lam, eta, alpha,
                                                 sigma0, max_n);
    return hipGetLastError();
}

}  // namespace qpa
