// Relaxed PA (analog spins in the target part, s := x) and its reverse-mode adjoint, for
// one instance or a batch of instances sharing the dynamics parameters.
//
// Forward step t of one element (FP32, each operation rounded separately):
//   f = (J x_t)_i;  h = f + b_i;  g = lambda_t x + h;  m' = alpha m - eta g;
//   y = x + m';  x' = clip(y, -1, 1).
// Loss: L = scale * sum over instances and replicas of [ (1/2) x_T^T J x_T + b^T x_T ].
// Reverse, with mu_{T+1} = 0 and xbar_T = scale (J x_T + b):
//   A(t):  ybar = xbar_{t+1} * [|y_{t+1}| <= 1];  mu_{t+1} = ybar + alpha mu_{t+2};
//          dL/deta += <mu, -g_t>,  dL/dalpha += <mu, m_t>,  dL/dlambda_t = <mu, -eta x_t>
//   B(t):  xbar_t = ybar - eta (lambda_t mu_{t+1} + J mu_{t+1})
// A needs only the element's own values; B needs J mu, a product over neighbours.  A step
// of the reverse pass is one launch that runs B(t) and then A(t-1) on each element ("BA"),
// with mu double-buffered since neighbours read it; a segment's first step runs A alone
// and its last B alone, because the state of the step before a segment is recomputed
// only with the next segment.
//
// State: every vector is [rows][Rp] FP32 (replica fastest); instance k of a batch owns the
// global rows [row0_k, row0_k + n_k).  Replicas r >= R are padding: held at zero and left
// out of every sum.
// Products with J: CSR couplings through row launches over blocks of 64 rows, the input
// vector staged through LDS (a wave = four rows and 64 replicas, lane = replica, each
// row's entries walked in order); dense FP32 couplings through the LDS-tiled product
// shared with the SBM step, with the element work in its epilogue.  Both add one fused multiply-add
// per term in ascending column order.
// Inner products are accumulated in FP64 per thread, reduced per workgroup in a fixed
// order and written to a per-step table of partial sums, which one last launch reduces in
// a fixed order: results do not depend on the checkpoint interval or on timing.
#include "fp32_tiled.h"
#include <type_traits>

namespace qpa {
namespace {

constexpr int REL_FWD = REL_MODE_FWD, REL_LOSS = REL_MODE_LOSS, REL_A = REL_MODE_A,
              REL_B = REL_MODE_B, REL_BA = REL_MODE_BA;

__device__ __forceinline__ void rel_fwd_point(float f, float bi, float lt, float eta,
                                              float alpha, float &x, float &m) {
    const float h = __fadd_rn(f, bi);
    const float g = __fadd_rn(__fmul_rn(lt, x), h);
    const float mn = __fsub_rn(__fmul_rn(alpha, m), __fmul_rn(eta, g));
    x = fminf(1.0f, fmaxf(-1.0f, __fadd_rn(x, mn)));
    m = mn;
}

// A(t) on one element from its stored state (x_t, m_t, f_t): the same FP32 operations as
// the forward step rebuild g_t and y_{t+1}.
__device__ __forceinline__ void rel_a_point(float x, float m, float f, float bi, float lt,
                                            float eta, float alpha, float xbar_next,
                                            float mu_next2, float &mu, float &yb, double &se,
                                            double &sa, double &sl) {
    const float h = __fadd_rn(f, bi);
    const float g = __fadd_rn(__fmul_rn(lt, x), h);
    const float mn = __fsub_rn(__fmul_rn(alpha, m), __fmul_rn(eta, g));
    const float y = __fadd_rn(x, mn);
    yb = fabsf(y) <= 1.0f ? xbar_next : 0.0f;
    mu = __fadd_rn(yb, __fmul_rn(alpha, mu_next2));
    se += (double)mu * (double)(-g);
    sa += (double)mu * (double)m;
    sl += (double)mu * (-(double)eta * (double)x);
}

__device__ __forceinline__ float rel_b_point(float yb, float mu, float jmu, float lt, float eta) {
    return __fsub_rn(yb, __fmul_rn(eta, __fadd_rn(__fmul_rn(lt, mu), jmu)));
}

__device__ __forceinline__ double rel_wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Fixed-order sum over the workgroup's waves (nw of them), result in thread 0.
__device__ __forceinline__ double rel_group_sum(double v, double *sh, int nw) {
    v = rel_wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < nw; ++k) s += sh[k];
    return s;
}

// Element work of one launch; `acc` is the product (J v)_i when the mode has one.
template <int MODE>
__device__ __forceinline__ void rel_element(const RelArgs &a, int64_t idx, bool live, float acc,
                                            float bi, double &s0, double &s1, double &s2) {
    if (MODE == REL_FWD) {
        float x = 0.0f, m = 0.0f;
        if (live) {
            x = a.xi[idx];
            m = a.mi[idx];
            rel_fwd_point(acc, bi, a.lam[a.t_f], a.eta, a.alpha, x, m);
        }
        a.xo[idx] = x;
        a.mo[idx] = m;
        if (a.fo) a.fo[idx] = live ? acc : 0.0f;
    } else if (MODE == REL_LOSS) {
        float xb = 0.0f;
        if (live) {
            const double x = a.xi[idx], f = acc, b = bi;
            s0 += 0.5 * x * f + b * x;
            xb = (float)(a.scale * (f + b));
        }
        a.xbar[idx] = xb;
    } else {
        float xbar_next = 0.0f;
        if (MODE == REL_A) {
            xbar_next = a.xbar[idx];
        } else {
            // B of the previous launch's step: xbar_t from ybar, mu_{t+1} and J mu_{t+1}
            const float xb = live ? rel_b_point(a.yb[idx], a.mu_in[idx], acc, a.lam[a.t_f],
                                                a.eta)
                                  : 0.0f;
            if (MODE == REL_B) {
                a.xbar[idx] = xb;
                return;
            }
            xbar_next = xb;
        }
        float mu = 0.0f, yb = 0.0f;
        if (live)
            rel_a_point(a.sx[idx], a.sm[idx], a.sf[idx], bi, a.lam[a.t_a], a.eta, a.alpha,
                        xbar_next, a.mu_in[idx], mu, yb, s0, s1, s2);
        a.mu_out[idx] = mu;
        a.yb[idx] = yb;
    }
}

// Writes this workgroup's partial sums (thread 0 holds the group sums).
template <int MODE>
__device__ __forceinline__ void rel_write_partials(const RelArgs &a, int64_t wg, double s0,
                                                   double s1, double s2, double *sh, int nw) {
    if (MODE == REL_FWD || MODE == REL_B) return;
    const double g0 = rel_group_sum(s0, sh, nw);
    if (MODE == REL_LOSS) {
        if (threadIdx.x == 0) a.part[a.slot0 + wg] = g0 * a.scale;
        return;
    }
    const double g1 = rel_group_sum(s1, sh, nw);
    const double g2 = rel_group_sum(s2, sh, nw);
    if (threadIdx.x == 0) {
        a.part[a.slot0 + wg] = g0;
        a.part[a.nblk + a.slot0 + wg] = g1;
        a.part[2 * a.nblk + a.slot0 + wg] = g2;
    }
}

template <typename T> __device__ __forceinline__ float as_weight(T w) { return (float)w; }

// Row launches: the CSR product with its input staged through LDS (the gather modes), and
// the element-wise pass (REL_A) over every instance's rows with the same work items, so
// that a step's partial sums are grouped alike whichever launch computes them.  Work item
// = (block of 64 consecutive rows of one instance, 64-replica chunk c); a workgroup of 16
// waves takes its items in the order below.  Wave w owns rows 4w .. 4w + 3 of the block
// (lane = replica) and keeps their running sums; the input vector (x or mu of the
// instance, the chunk's 64 replicas) goes through LDS 256 columns at a time (one buffer of
// 64 KiB: a range is staged, then walked; the other workgroup on the compute unit walks
// while this one stages), and each row walks its entries
// whose column falls in the staged range, in ascending order, one fused multiply-add per
// term (the order of the definition), while each staged value serves all 64 rows of the
// block instead of one gather per entry.  A row's entries come in windows of 64 (lane k =
// entry k past the row's cursor).  At the start of a range the number of each row's
// entries in it is counted from the window at hand; the windows past them (all four rows)
// are loaded into a second register set before any row is walked, so that they are in
// flight during the walks, and they are converted only when the next range counts them.
// The loads are issued without per-lane branches.
typedef __attribute__((address_space(3))) void lds_void;
constexpr int GR_THREADS = 1024, GR_WAVES = GR_THREADS / 64, GR_RPW = 4;
constexpr int GR_ROWS = GR_WAVES * GR_RPW;       // 64 rows per block
constexpr int GR_CW = 256;                       // staged columns per range
static_assert(GR_ROWS == 64, "blocks of 64 rows");

typedef const __attribute__((address_space(1))) int32_t *gr_i32;

// A row's window as loaded (raw column and weight of entry cursor + lane; lanes past the
// row's end hold some stored entry of the instance); converted when it is used, so that
// its loads stay in flight until then.
template <typename TW, typename TI> struct GrWin {
    TI j[GR_RPW];
    TW w[GR_RPW];
};

// Two workgroups per CU (64 KiB of LDS each, 8 waves per SIMD): the walks are bound by
// the latency of their LDS reads, which the second workgroup's waves hide, as they hide
// each range's staging.
template <int MODE, typename TW, typename TI>
__global__ void __launch_bounds__(GR_THREADS)
    __attribute__((amdgpu_waves_per_eu(8))) k_rel_gather(const RelInst *__restrict__ insts,
                                                           int32_t ninst, int64_t blocks,
                                                           int32_t C, const RelArgs a) {
    constexpr bool GATHER = MODE != REL_A;
    typedef const __attribute__((address_space(1))) TW *gw_t;
    typedef const __attribute__((address_space(1))) TI *gi_t;
    __shared__ __attribute__((aligned(16))) float vs[GATHER ? GR_CW * 64 : 1];
    __shared__ double sh[GR_WAVES];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    const int64_t total = blocks * C;
    // items in chunks of P = (workgroups / 8) consecutive ones, chunk k on compute die
    // k mod 8 (workgroup b runs on die b mod 8): the items a die runs at a time are
    // neighbouring blocks, mostly of one instance, whose input vector its L2 then holds
    // for all of them instead of every die fetching every instance's
    const int64_t P = gridDim.x >> 3;
    const int64_t die = blockIdx.x & 7, slot = blockIdx.x >> 3;
    for (int64_t k = die; k * P + slot < total; k += 8) {
        const int64_t it = k * P + slot;
        const int64_t blk = it / C;
        const int c = (int)(it - blk * C);
        int lo = 0, hi = ninst - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (insts[mid].blk0 <= blk) lo = mid;
            else hi = mid - 1;
        }
        // the instance's fields, read once (a staging load may write memory as far as the
        // compiler knows, which would otherwise make it read them again)
        const RelInst &I = insts[lo];
        const int64_t n = I.n;
        const int64_t i0 = (blk - I.blk0) * GR_ROWS + GR_RPW * wv;
        float acc[GR_RPW];
#pragma unroll
        for (int u = 0; u < GR_RPW; ++u) acc[u] = 0.0f;
        if (GATHER) {
            const gr_i32 rp = (gr_i32)I.rp;
            const int32_t rp0 = rp[0];
            // (an instance without stored entries has nothing to gather: uniform per item)
            if (rp[n] > rp0) {
                const float *v = ((MODE == REL_FWD || MODE == REL_LOSS) ? a.xi : a.mu_in) +
                                 I.row0 * a.Rp + (int64_t)c * 64;
                const gi_t col = (gi_t)I.col;
                const gw_t w = (gw_t)I.w;
                const bool skip = I.skip_diag != 0;
                // staging of columns GR_CW q .. GR_CW q + GR_CW - 1 (past n: column n - 1
                // again, unused): thread t moves GR_CW / 64 pieces of 16 bytes, element
                // e = 1024 u + t = column e / 16 of the range, floats 4 (e % 16) .. + 3; a
                // wave's destinations are contiguous.  Addresses are the range's uniform
                // base plus 32-bit offsets.
                const uint32_t rp4 = (uint32_t)a.Rp;
                auto stage = [&](int q) {
                    const float *vq = v + (int64_t)q * GR_CW * a.Rp;
                    const uint32_t lim =
                        (uint32_t)min((int64_t)GR_CW - 1, n - 1 - (int64_t)q * GR_CW);
#pragma unroll
                    for (int u = 0; u < GR_CW / 64; ++u) {
                        const uint32_t e = 1024u * u + threadIdx.x;
                        const uint32_t o = __umul24(min(e >> 4, lim), rp4) + 4u * (e & 15u);
                        __builtin_amdgcn_global_load_lds(
                            vq + o, (lds_void *)(vs + 4 * (1024 * u + 64 * wv)), 16, 0, 0);
                    }
                };
                int32_t kc[GR_RPW], ke[GR_RPW];
#pragma unroll
                for (int u = 0; u < GR_RPW; ++u) {
                    const int64_t i = i0 + u;
                    kc[u] = i < n ? rp[i] : rp0;
                    ke[u] = i < n ? rp[i + 1] : rp0;
                }
                // row u's window from its cursor kc[u] (two loads, no branch)
                auto load = [&](GrWin<TW, TI> &W, int u) {
                    const int32_t kk = min(kc[u] + lane, max(ke[u] - 1, rp0));
                    W.j[u] = col[kk];
                    W.w[u] = w[kk];
                };
                // its entries as columns (past the row's end: one no range reaches) and
                // weights (a stored QUBO diagonal is folded into b: weight 0 adds nothing)
                auto cols = [&](const GrWin<TW, TI> &W, int u) {
                    return kc[u] + lane < ke[u] ? (int32_t)W.j[u] : INT32_MAX;
                };
                auto weights = [&](const GrWin<TW, TI> &W, int u) {
                    const float wf = as_weight(W.w[u]);
                    return skip && (int64_t)W.j[u] == i0 + u ? 0.0f : wf;
                };
                auto walk = [&](int32_t jl, float wl, int u, int cnt, int32_t base,
                                const float *src) {
                    int e = 0;
                    const int wi = __float_as_int(wl);
                    for (; e + 4 <= cnt; e += 4) {
                        const int32_t j0 = __builtin_amdgcn_readlane(jl, e) - base;
                        const int32_t j1 = __builtin_amdgcn_readlane(jl, e + 1) - base;
                        const int32_t j2 = __builtin_amdgcn_readlane(jl, e + 2) - base;
                        const int32_t j3 = __builtin_amdgcn_readlane(jl, e + 3) - base;
                        const float v0 = src[64 * j0], v1 = src[64 * j1];
                        const float v2 = src[64 * j2], v3 = src[64 * j3];
                        acc[u] = __fmaf_rn(__int_as_float(__builtin_amdgcn_readlane(wi, e)),
                                           v0, acc[u]);
                        acc[u] = __fmaf_rn(
                            __int_as_float(__builtin_amdgcn_readlane(wi, e + 1)), v1, acc[u]);
                        acc[u] = __fmaf_rn(
                            __int_as_float(__builtin_amdgcn_readlane(wi, e + 2)), v2, acc[u]);
                        acc[u] = __fmaf_rn(
                            __int_as_float(__builtin_amdgcn_readlane(wi, e + 3)), v3, acc[u]);
                    }
                    for (; e < cnt; ++e) {
                        const int32_t j = __builtin_amdgcn_readlane(jl, e) - base;
                        acc[u] = __fmaf_rn(__int_as_float(__builtin_amdgcn_readlane(wi, e)),
                                           src[64 * j], acc[u]);
                    }
                };
                // Integer weights of 8 or 16 bits: the float of such a weight has its low 8
                // bits zero, which then carry the entry's column within the staged range,
                // so that one read of the window word gives both (the column on the scalar
                // unit, the weight as it is).
                constexpr bool PACK = std::is_integral<TW>::value && sizeof(TW) <= 2;
                // Two forms of the word: 8-bit weights' floats have their low 16 bits zero
                // too, which then carry the column's byte offset in the staged range as it is
                // (one AND on the scalar unit instead of a shift and an AND); other 8- or
                // 16-bit weights carry the column index in their low 8 bits.  W16 (a
                // compile-time tag) selects the form.
                auto pack = [&](int32_t jl, float wl, int32_t base, auto w16) {
                    if (decltype(w16)::value)
                        return (__float_as_int(wl) & (int32_t)0xFFFF0000) |
                               (((jl - base) & 0xFF) << 8);
                    return (__float_as_int(wl) & ~0xFF) | ((jl - base) & 0xFF);
                };
                auto offs = [](int32_t p, auto w16) -> int32_t {
                    return decltype(w16)::value ? (p & 0xFF00) : ((p & 0xFF) << 8);
                };
                auto wgt = [](int32_t p, auto w16) -> float {
                    return __int_as_float(decltype(w16)::value ? (p & (int32_t)0xFFFF0000)
                                                               : (p & ~0xFF));
                };
                // the staged value of a word's column for this lane's replica
                auto val = [&](const float *src, int32_t p, auto w16) {
                    return *reinterpret_cast<const float *>(
                        reinterpret_cast<const char *>(src) + offs(p, w16));
                };
                auto walkp = [&](int32_t pk, int u, int e, int cnt, const float *src, auto w16) {
                    for (; e + 4 <= cnt; e += 4) {
                        const int32_t p0 = __builtin_amdgcn_readlane(pk, e);
                        const int32_t p1 = __builtin_amdgcn_readlane(pk, e + 1);
                        const int32_t p2 = __builtin_amdgcn_readlane(pk, e + 2);
                        const int32_t p3 = __builtin_amdgcn_readlane(pk, e + 3);
                        const float v0 = val(src, p0, w16), v1 = val(src, p1, w16);
                        const float v2 = val(src, p2, w16), v3 = val(src, p3, w16);
                        acc[u] = __fmaf_rn(wgt(p0, w16), v0, acc[u]);
                        acc[u] = __fmaf_rn(wgt(p1, w16), v1, acc[u]);
                        acc[u] = __fmaf_rn(wgt(p2, w16), v2, acc[u]);
                        acc[u] = __fmaf_rn(wgt(p3, w16), v3, acc[u]);
                    }
                    for (; e < cnt; ++e) {
                        const int32_t p = __builtin_amdgcn_readlane(pk, e);
                        acc[u] = __fmaf_rn(wgt(p, w16), val(src, p, w16), acc[u]);
                    }
                };
                // rows u and u + 1 together over their common first entries (eight reads in
                // flight, two independent sums), then each alone
                auto walkp2 = [&](int32_t pa, int32_t pb, int u, int ca, int cb,
                                  const float *src, auto w16) {
                    const int cm = min(ca, cb);
                    int e = 0;
                    for (; e + 4 <= cm; e += 4) {
                        int32_t p[8];
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            p[k] = __builtin_amdgcn_readlane(pa, e + k);
                            p[4 + k] = __builtin_amdgcn_readlane(pb, e + k);
                        }
                        float vv[8];
#pragma unroll
                        for (int k = 0; k < 8; ++k) vv[k] = val(src, p[k], w16);
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            acc[u] = __fmaf_rn(wgt(p[k], w16), vv[k], acc[u]);
                            acc[u + 1] = __fmaf_rn(wgt(p[4 + k], w16), vv[4 + k], acc[u + 1]);
                        }
                    }
                    walkp(pa, u, e, ca, src, w16);
                    walkp(pb, u + 1, e, cb, src, w16);
                };
                auto walk_any = [&](int32_t jl, float wl, int u, int cnt, int32_t base,
                                    const float *src) {
                    if (PACK) walkp(pack(jl, wl, base, std::false_type{}), u, 0, cnt, src,
                                    std::false_type{});
                    else walk(jl, wl, u, cnt, base, src);
                };
                const int nq = (int)((n + GR_CW - 1) / GR_CW);
                GrWin<TW, TI> A, B;
#pragma unroll
                for (int u = 0; u < GR_RPW; ++u) load(A, u);
                // range q: load Y (the windows past this range's entries of every row),
                // then walk X (the windows at the cursors before)
                auto range = [&](int q, GrWin<TW, TI> &X, GrWin<TW, TI> &Y) {
                    // every wave is done with range q - 1, then the buffer takes range q
                    // and every wave's part has landed
                    if (q > 0) asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
                    stage(q);
                    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
                    const int32_t base = q * GR_CW, bound = base + GR_CW;
                    int32_t jl[GR_RPW];
                    float wl[GR_RPW];
                    int cnt[GR_RPW];
#pragma unroll
                    for (int u = 0; u < GR_RPW; ++u) {
                        jl[u] = cols(X, u);
                        wl[u] = weights(X, u);
                        cnt[u] = __popcll(__ballot(jl[u] < bound));
                    }
                    const float *src = vs + lane;
#pragma unroll
                    for (int u = 0; u < GR_RPW; ++u) {
                        kc[u] += cnt[u];
                        load(Y, u);
                    }
                    if (PACK) {
                        // the 16-bit form when every weight of the four windows fits it
                        bool w16 = true;
#pragma unroll
                        for (int u = 0; u < GR_RPW; ++u)
                            w16 = w16 && __ballot(kc[u] - cnt[u] + lane < ke[u] &&
                                                  fabsf(wl[u]) > 255.0f) == 0;
                        if (w16) {
#pragma unroll
                            for (int u = 0; u < GR_RPW; u += 2)
                                walkp2(pack(jl[u], wl[u], base, std::true_type{}),
                                       pack(jl[u + 1], wl[u + 1], base, std::true_type{}), u,
                                       cnt[u], cnt[u + 1], src, std::true_type{});
                        } else {
#pragma unroll
                            for (int u = 0; u < GR_RPW; u += 2)
                                walkp2(pack(jl[u], wl[u], base, std::false_type{}),
                                       pack(jl[u + 1], wl[u + 1], base, std::false_type{}), u,
                                       cnt[u], cnt[u + 1], src, std::false_type{});
                        }
                    }
#pragma unroll
                    for (int u = 0; u < GR_RPW; ++u) {
                        if (!PACK) walk_any(jl[u], wl[u], u, cnt[u], base, src);
                        if (cnt[u] == 64) {
                            // more of the row's entries in this range (rare): walk on from
                            // Y, which starts at the cursor, and reload it after them
                            for (;;) {
                                const int32_t j2 = cols(Y, u);
                                const int c2 = __popcll(__ballot(j2 < bound));
                                walk_any(j2, weights(Y, u), u, c2, base, src);
                                kc[u] += c2;
                                load(Y, u);
                                if (c2 < 64) break;
                            }
                        }
                    }
                };
                int q = 0;
                for (; q + 2 <= nq; q += 2) {
                    range(q, A, B);
                    range(q + 1, B, A);
                }
                if (q < nq) range(q, A, B);
                // every wave is done with the staging buffers before the next item loads
                // them
                __syncthreads();
            }
        }
        const int64_t r = (int64_t)c * 64 + lane;
#pragma unroll
        for (int u = 0; u < GR_RPW; ++u) {
            const int64_t i = i0 + u;
            if (i < n)
                rel_element<MODE>(a, (I.row0 + i) * a.Rp + r, r < a.R, acc[u], I.b[i], s0, s1,
                                  s2);
        }
    }
    rel_write_partials<MODE>(a, blockIdx.x, s0, s1, s2, sh, GR_WAVES);
}

// Epilogue of the dense tiled product for every mode (b, and the state pointers in `a`,
// already offset to the instance's rows).
template <int MODE>
struct RelTileEpilogue {
    RelArgs a;
    const float *b;
    __device__ __forceinline__ void operator()(float (&acc)[8][8], int64_t n, int64_t Rp,
                                               int64_t i0, int64_t r0, int tx, int ty) const {
        __shared__ double sh[4];
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int64_t i = i0 + 64 * (v >> 2) + 4 * tx + (v & 3);
            if (i >= n) continue;
            const float bi = b[i];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t r = r0 + 64 * h + 4 * ty + e;
                    rel_element<MODE>(a, i * Rp + r, r < a.R, acc[4 * h + e][v], bi, s0, s1,
                                      s2);
                }
        }
        rel_write_partials<MODE>(a, (int64_t)blockIdx.y * gridDim.x + blockIdx.x, s0, s1, s2,
                                 sh, 4);
    }
};

__global__ void __launch_bounds__(256) k_rel_fill(double *__restrict__ p, int64_t count) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count;
         q += (int64_t)gridDim.x * blockDim.x)
        p[q] = 0.0;
}

// Final reduction of the per-step partial tables, in a fixed order: thread t sums the
// slots of steps t, t + 256, ... (d_lambda_t, and the step's d_eta and d_alpha terms,
// which it leaves in the step's first slots), then thread 0 sums the steps in order.
__global__ void __launch_bounds__(256) k_rel_finish(int32_t T, int32_t nblk,
                                                    double *__restrict__ part_steps,
                                                    const double *__restrict__ part_loss,
                                                    double *__restrict__ loss,
                                                    double *__restrict__ d_eta,
                                                    double *__restrict__ d_alpha,
                                                    double *__restrict__ d_lam) {
    const bool grads = d_eta || d_alpha || d_lam;
    if (grads)
        for (int32_t t = threadIdx.x; t < T; t += blockDim.x) {
            double *p = part_steps + (int64_t)t * 3 * nblk;
            double e = 0.0, a = 0.0, l = 0.0;
            for (int32_t k = 0; k < nblk; ++k) {
                e += p[k];
                a += p[nblk + k];
                l += p[2 * nblk + k];
            }
            p[0] = e;
            p[nblk] = a;
            if (d_lam) d_lam[t] = l;
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        double L = 0.0;
        for (int32_t k = 0; k < nblk; ++k) L += part_loss[k];
        *loss = L;
        if (grads) {
            double e = 0.0, a = 0.0;
            for (int32_t t = 0; t < T; ++t) {
                e += part_steps[(int64_t)t * 3 * nblk];
                a += part_steps[(int64_t)t * 3 * nblk + nblk];
            }
            if (d_eta) *d_eta = e;
            if (d_alpha) *d_alpha = a;
        }
    }
}

template <typename F>
hipError_t rel_by_dtypes(int32_t wdt, int32_t idt, F &&f) {
    auto byw = [&](auto itag) -> hipError_t {
        switch (wdt) {
            case QPA_I8: return f((int8_t)0, itag);
            case QPA_I16: return f((int16_t)0, itag);
            case QPA_I32: return f((int32_t)0, itag);
            default: return f(0.0f, itag);
        }
    };
    return idt == QPA_I16 ? byw((int16_t)0) : byw((int32_t)0);
}

template <int MODE>
hipError_t rel_gather_launch(const RelInst *insts, int32_t ninst, int64_t blocks, int32_t C,
                             int32_t wdt, int32_t idt, const RelArgs &a, hipStream_t st) {
    const unsigned g = (unsigned)rel_gather_blocks(blocks, C);
    if (g % 8) return hipErrorInvalidValue;       // the item order assumes whole dies
    if (MODE == REL_A) {
        k_rel_gather<REL_A, float, int32_t><<<g, GR_THREADS, 0, st>>>(insts, ninst, blocks, C, a);
        return hipGetLastError();
    }
    return rel_by_dtypes(wdt, idt, [&](auto wtag, auto itag) {
        using TW = decltype(wtag);
        using TI = decltype(itag);
        k_rel_gather<MODE, TW, TI><<<g, GR_THREADS, 0, st>>>(insts, ninst, blocks, C, a);
        return hipGetLastError();
    });
}

template <int MODE>
hipError_t rel_tile_launch(int64_t n, const float *J, const float *b, const RelArgs &a,
                           hipStream_t st) {
    if (a.Rp % SB_BR || n < 1) return hipErrorInvalidValue;
    dim3 grid((unsigned)((n + SB_BI - 1) / SB_BI), (unsigned)(a.Rp / SB_BR));
    const RelTileEpilogue<MODE> epi{a, b};
    const float *q = (MODE == REL_FWD || MODE == REL_LOSS) ? a.xi : a.mu_in;
    if (n % 4 == 0)
        k_fp32_tiled_step<true, RelTileEpilogue<MODE>><<<grid, 256, 0, st>>>(n, a.Rp, J, q, epi);
    else
        k_fp32_tiled_step<false, RelTileEpilogue<MODE>><<<grid, 256, 0, st>>>(n, a.Rp, J, q, epi);
    return hipGetLastError();
}

}  // namespace

int64_t rel_gather_blocks(int64_t blocks, int32_t C) {
    int64_t g = (blocks * (int64_t)C + 7) / 8 * 8;          // a multiple of the 8 dies
    if (g > REL_GATHER_BLOCKS_MAX) g = REL_GATHER_BLOCKS_MAX;
    return g < 8 ? 8 : g;
}

hipError_t launch_rel_gather(int32_t mode, const RelInst *insts, int32_t ninst, int64_t blocks,
                             int32_t C, int32_t wdt, int32_t idt, const RelArgs &a,
                             hipStream_t st) {
    switch (mode) {
        case REL_FWD: return rel_gather_launch<REL_FWD>(insts, ninst, blocks, C, wdt, idt, a, st);
        case REL_LOSS: return rel_gather_launch<REL_LOSS>(insts, ninst, blocks, C, wdt, idt, a, st);
        case REL_A: return rel_gather_launch<REL_A>(insts, ninst, blocks, C, wdt, idt, a, st);
        case REL_B: return rel_gather_launch<REL_B>(insts, ninst, blocks, C, wdt, idt, a, st);
        case REL_BA: return rel_gather_launch<REL_BA>(insts, ninst, blocks, C, wdt, idt, a, st);
    }
    return hipErrorInvalidValue;
}

int64_t rel_tile_blocks(int64_t n, int64_t Rp) {
    return ((n + SB_BI - 1) / SB_BI) * (Rp / SB_BR);
}

hipError_t launch_rel_tiles(int32_t mode, int64_t n, const float *J, const float *b,
                            const RelArgs &a, hipStream_t st) {
    switch (mode) {
        case REL_FWD: return rel_tile_launch<REL_FWD>(n, J, b, a, st);
        case REL_LOSS: return rel_tile_launch<REL_LOSS>(n, J, b, a, st);
        case REL_B: return rel_tile_launch<REL_B>(n, J, b, a, st);
        case REL_BA: return rel_tile_launch<REL_BA>(n, J, b, a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_rel_fill(double *p, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t g = (count + 255) / 256;
    if (g > 1024) g = 1024;
    k_rel_fill<<<(unsigned)g, 256, 0, st>>>(p, count);
    return hipGetLastError();
}

hipError_t launch_rel_finish(int32_t T, int32_t nblk, double *part_steps,
                             const double *part_loss, double *loss, double *d_eta,
                             double *d_alpha, double *d_lam, hipStream_t st) {
    k_rel_finish<<<1, 256, 0, st>>>(T, nblk, part_steps, part_loss, loss, d_eta, d_alpha, d_lam);
    return hipGetLastError();
}

}  // namespace qpa
