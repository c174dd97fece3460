// C ABI of libqpa: argument checks, workspace planning and the order of launches of a
// solve.  Every step of the method runs in the kernels of the other translation units.
#include "qpa_internal.h"

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

struct qpa_ctx {
    int device = 0;
    std::string err;
    int32_t *host_flags = nullptr;          // pinned, for the validation read-back
    qpa::CanonScalars *host_sc = nullptr;   // pinned
    float *host_lam = nullptr;              // pinned schedule staging
    size_t host_lam_cap = 0;
    // step-kernel timing (qpa_profile_*)
    bool prof = false;
    struct Span {
        hipEvent_t a, b;
        int64_t launches;
    };
    std::vector<Span> spans;
    std::vector<hipEvent_t> free_events;
};

namespace qpa {
namespace {

constexpr size_t ALIGN = 256;

inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }
inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

enum class Path { DenseResident, DenseTiled, DenseMfma, Csr };

const char *path_name(Path p) {
    switch (p) {
        case Path::DenseResident: return "dense-resident-fp32";
        case Path::DenseTiled: return "dense-tiled-fp32";
        case Path::DenseMfma: return "dense-mfma-bf16";
        case Path::Csr: return "csr";
    }
    return "?";
}

struct Plan {
    Path path;
    int64_t n, R, T;
    int64_t np, Rp;       // padded sizes of the internal state
    int G;                // CSR replica group
    int64_t nwords;       // CSR spin words per group
    bool is_int, is_qubo;
    int64_t eblk;         // energy partial blocks
    // workspace offsets (bytes)
    size_t o_sc, o_lam, o_bf, o_bi, o_bd, o_rabs, o_rmax, o_rk, o_Jf, o_Jb, o_x, o_m, o_h,
        o_s0, o_s1, o_part, o_ei, o_ed, o_sp, o_best, total;
};

int64_t energy_blocks(const qpa_problem &p) {
    return p.format == QPA_FMT_DENSE ? (p.n + 3) / 4 : (p.n + 255) / 256;
}

Plan make_plan(const qpa_problem &p, const qpa_params &a) {
    Plan pl{};
    pl.n = p.n;
    pl.R = a.replicas;
    pl.T = a.steps;
    pl.is_int = dtype_is_int(p.coupling_dtype) &&
                (p.linear == nullptr || dtype_is_int(p.linear_dtype));
    pl.is_qubo = p.kind == QPA_KIND_QUBO;
    pl.np = pl.n;
    pl.Rp = pl.R;
    pl.G = 1;
    pl.nwords = 0;
    if (p.format == QPA_FMT_CSR) {
        pl.path = Path::Csr;
        pl.G = csr_group_size(pl.R);
        pl.Rp = round_up(pl.R, pl.G);
        pl.nwords = csr_words_per_group(pl.n, pl.G);
    } else if (a.precision == QPA_PREC_BF16) {
        pl.path = Path::DenseMfma;
        pl.np = round_up(pl.n, std::max(MF_BN, MF_BK));
        pl.Rp = round_up(pl.R, MF_BM);
    } else if (dense_resident_fits(pl.n)) {
        pl.path = Path::DenseResident;
    } else {
        pl.path = Path::DenseTiled;
    }
    pl.eblk = energy_blocks(p);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes);
        return o;
    };
    const size_t n = (size_t)pl.n, np = (size_t)pl.np, R = (size_t)pl.R, Rp = (size_t)pl.Rp;
    pl.o_sc = take(sizeof(CanonScalars));
    pl.o_lam = take(sizeof(float) * (size_t)std::max<int64_t>(pl.T, 1));
    pl.o_bf = take(sizeof(float) * np);
    pl.o_bi = take(sizeof(int64_t) * n);
    pl.o_bd = take(sizeof(double) * n);
    pl.o_rabs = take(sizeof(double) * n);
    pl.o_rmax = take(sizeof(double) * n);
    pl.o_rk = take(sizeof(double) * n);
    pl.o_Jf = (pl.path == Path::DenseResident || pl.path == Path::DenseTiled)
                  ? take(sizeof(float) * n * n) : 0;
    pl.o_Jb = pl.path == Path::DenseMfma ? take(sizeof(uint16_t) * np * np) : 0;
    pl.o_x = take(sizeof(float) * Rp * np);
    pl.o_m = take(sizeof(float) * Rp * np);
    pl.o_h = take(sizeof(float) * Rp * np);
    size_t sbytes = 0;
    switch (pl.path) {
        case Path::DenseResident: sbytes = 0; break;
        case Path::DenseTiled: sbytes = sizeof(float) * R * n; break;
        case Path::DenseMfma: sbytes = sizeof(uint32_t) * Rp * (np / 32); break;
        case Path::Csr: sbytes = sizeof(uint64_t) * (size_t)(Rp / pl.G) * (size_t)pl.nwords; break;
    }
    pl.o_s0 = sbytes ? take(sbytes) : 0;
    pl.o_s1 = sbytes ? take(sbytes) : 0;
    pl.o_part = take(sizeof(double) * (size_t)pl.eblk * R);
    pl.o_ei = take(sizeof(int64_t) * R);
    pl.o_ed = take(sizeof(double) * R);
    pl.o_sp = take(sizeof(int8_t) * R * n);
    pl.o_best = take(sizeof(int32_t) * 4);
    pl.total = off;
    return pl;
}

// Strides of element (r, i) in the internal state layout of a plan.
void state_strides(const Plan &pl, int64_t &ld_r, int64_t &ld_i) {
    if (pl.path == Path::Csr) {
        ld_r = 1;
        ld_i = pl.Rp;
    } else {
        ld_r = pl.np;
        ld_i = 1;
    }
}

// Message of the last failure of a call made without a context (per host thread).
thread_local std::string g_noctx_err;

qpa_status fail(qpa_ctx *ctx, qpa_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_noctx_err = buf;
    return s;
}

#define QPA_HIP(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(ctx, QPA_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

bool dtype_ok(int32_t dt) { return dt >= QPA_I8 && dt <= QPA_F32; }

qpa_status check_problem(qpa_ctx *ctx, const qpa_problem *p) {
    if (!p) return fail(ctx, QPA_E_ARG, "problem is NULL");
    if (p->n < 1) return fail(ctx, QPA_E_SHAPE, "n must be >= 1 (got %lld)", (long long)p->n);
    if (p->kind != QPA_KIND_QUBO && p->kind != QPA_KIND_ISING)
        return fail(ctx, QPA_E_ARG, "unknown problem kind %d", p->kind);
    if (!dtype_ok(p->coupling_dtype))
        return fail(ctx, QPA_E_ARG, "unknown coupling dtype %d", p->coupling_dtype);
    if (p->linear && !dtype_ok(p->linear_dtype))
        return fail(ctx, QPA_E_ARG, "unknown linear dtype %d", p->linear_dtype);
    if (p->format == QPA_FMT_DENSE) {
        if (!p->dense) return fail(ctx, QPA_E_ARG, "dense couplings pointer is NULL");
        if (p->n > 262144) return fail(ctx, QPA_E_SHAPE, "dense n too large");
    } else if (p->format == QPA_FMT_CSR) {
        if (!p->row_ptr || (p->nnz > 0 && (!p->col || !p->weights)))
            return fail(ctx, QPA_E_ARG, "CSR pointer is NULL");
        if (p->nnz < 0 || p->nnz >= ((int64_t)1 << 31))
            return fail(ctx, QPA_E_SHAPE, "nnz out of range for int32 row pointers");
        if (p->index_dtype != QPA_I32 && p->index_dtype != QPA_I16)
            return fail(ctx, QPA_E_ARG, "CSR index dtype must be I32 or I16");
        if (p->index_dtype == QPA_I16 && p->n > 32767)
            return fail(ctx, QPA_E_SHAPE, "int16 column indices need n <= 32767");
        if (p->n >= ((int64_t)1 << 31)) return fail(ctx, QPA_E_SHAPE, "n too large");
    } else {
        return fail(ctx, QPA_E_ARG, "unknown format %d", p->format);
    }
    return QPA_OK;
}

qpa_status check_params(qpa_ctx *ctx, const qpa_params *a) {
    if (!a) return fail(ctx, QPA_E_ARG, "params is NULL");
    if (a->replicas < 1) return fail(ctx, QPA_E_ARG, "replicas must be >= 1");
    if (a->steps < 0) return fail(ctx, QPA_E_ARG, "steps must be >= 0");
    if (a->precision != QPA_PREC_FP32 && a->precision != QPA_PREC_BF16)
        return fail(ctx, QPA_E_ARG, "unknown precision %d", a->precision);
    if (a->flags != 0) return fail(ctx, QPA_E_ARG, "params.flags must be 0");
    return QPA_OK;
}

template <typename T> T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// Schedule table (host, FP32, rounded as written) -> pinned staging -> workspace.
qpa_status upload_schedule(qpa_ctx *ctx, const qpa_params &a, float *d_lam, hipStream_t st) {
    const int64_t T = a.steps;
    if (T == 0) return QPA_OK;
    if (ctx->host_lam_cap < (size_t)T) {
        if (ctx->host_lam) (void)hipHostFree(ctx->host_lam);
        ctx->host_lam = nullptr;
        QPA_HIP(hipHostMalloc((void **)&ctx->host_lam, sizeof(float) * (size_t)T));
        ctx->host_lam_cap = (size_t)T;
    }
    // the staging buffer may still feed a copy of a previous call on this stream
    QPA_HIP(hipStreamSynchronize(st));
    for (int64_t t = 0; t < T; ++t) {
        if (a.lambda_table) {
            ctx->host_lam[t] = a.lambda_table[t];
        } else {
            volatile float frac = (float)t / (float)T;
            volatile float one_minus = 1.0f - frac;
            ctx->host_lam[t] = a.lambda0 * one_minus;
        }
    }
    QPA_HIP(hipMemcpyAsync(d_lam, ctx->host_lam, sizeof(float) * (size_t)T,
                           hipMemcpyHostToDevice, st));
    return QPA_OK;
}

// Canonicalise + validate; synchronises the stream to read the validation flags.
qpa_status canonicalise(qpa_ctx *ctx, const qpa_problem &p, const Plan &pl, void *ws,
                        hipStream_t st) {
    CanonScalars *sc = at<CanonScalars>(ws, pl.o_sc);
    float *bf = at<float>(ws, pl.o_bf);
    if (pl.np > pl.n) QPA_HIP(hipMemsetAsync(bf, 0, sizeof(float) * (size_t)pl.np, st));
    if (p.format == QPA_FMT_DENSE) {
        float *Jf = pl.o_Jf ? at<float>(ws, pl.o_Jf) : nullptr;
        uint16_t *Jb = pl.o_Jb ? at<uint16_t>(ws, pl.o_Jb) : nullptr;
        QPA_HIP(launch_canon_dense(p, Jf, Jb, pl.np, bf, at<int64_t>(ws, pl.o_bi),
                                   at<double>(ws, pl.o_bd), at<double>(ws, pl.o_rabs),
                                   at<double>(ws, pl.o_rmax), at<double>(ws, pl.o_rk), sc, st));
    } else {
        QPA_HIP(launch_canon_csr(p, bf, at<int64_t>(ws, pl.o_bi), at<double>(ws, pl.o_bd),
                                 at<double>(ws, pl.o_rabs), at<double>(ws, pl.o_rk), sc, st));
    }
    QPA_HIP(hipMemcpyAsync(ctx->host_sc, sc, sizeof(CanonScalars), hipMemcpyDeviceToHost, st));
    QPA_HIP(hipStreamSynchronize(st));
    const int32_t f = ctx->host_sc->flags;
    if (f & FLAG_SHAPE)
        return fail(ctx, QPA_E_SHAPE, "CSR row pointers or column indices are inconsistent");
    if (f & FLAG_UNSORTED)
        return fail(ctx, QPA_E_SHAPE, "CSR columns must be strictly increasing within a row");
    if (f & FLAG_ASYM)
        return fail(ctx, QPA_E_ASYM, p.kind == QPA_KIND_ISING
                                         ? "couplings not symmetric or Ising diagonal non-zero"
                                         : "couplings not symmetric");
    if (f & FLAG_RANGE)
        return fail(ctx, QPA_E_RANGE,
                    "integer row bound max_i sum_j |J_ij| + |b_i| = %.0f >= 2^24",
                    ctx->host_sc->max_row);
    return QPA_OK;
}

hipError_t take_event(qpa_ctx *ctx, hipEvent_t *ev) {
    if (!ctx->free_events.empty()) {
        *ev = ctx->free_events.back();
        ctx->free_events.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(ev);
}

qpa_status run_steps_inner(qpa_ctx *ctx, const qpa_problem &p, const qpa_params &a,
                           const Plan &pl, void *ws, int32_t t0, int32_t t1, bool want_h,
                           hipStream_t st, int64_t &launches);

// Run steps t0 .. t1-1 on the internal state of the plan (timed when profiling).
qpa_status run_steps(qpa_ctx *ctx, const qpa_problem &p, const qpa_params &a, const Plan &pl,
                     void *ws, int32_t t0, int32_t t1, bool want_h, hipStream_t st) {
    if (t1 <= t0) return QPA_OK;
    int64_t launches = 0;
    if (!ctx->prof) return run_steps_inner(ctx, p, a, pl, ws, t0, t1, want_h, st, launches);
    qpa_ctx::Span sp{};
    QPA_HIP(take_event(ctx, &sp.a));
    QPA_HIP(take_event(ctx, &sp.b));
    QPA_HIP(hipEventRecord(sp.a, st));
    qpa_status s = run_steps_inner(ctx, p, a, pl, ws, t0, t1, want_h, st, launches);
    QPA_HIP(hipEventRecord(sp.b, st));
    sp.launches = launches;
    ctx->spans.push_back(sp);
    return s;
}

qpa_status run_steps_inner(qpa_ctx *ctx, const qpa_problem &p, const qpa_params &a,
                           const Plan &pl, void *ws, int32_t t0, int32_t t1, bool want_h,
                           hipStream_t st, int64_t &launches) {
    float *x = at<float>(ws, pl.o_x), *m = at<float>(ws, pl.o_m);
    float *h = want_h ? at<float>(ws, pl.o_h) : nullptr;
    const float *lam = at<float>(ws, pl.o_lam);
    const float *bf = at<float>(ws, pl.o_bf);
    switch (pl.path) {
        case Path::DenseResident:
            QPA_HIP(launch_dense_resident(pl.n, pl.R, at<float>(ws, pl.o_Jf), bf, x, m, h, t0, t1,
                                          lam, a.eta, a.alpha, st));
            launches = 1;
            break;
        case Path::DenseTiled: {
            float *s0 = at<float>(ws, pl.o_s0), *s1 = at<float>(ws, pl.o_s1);
            QPA_HIP(launch_sign_f32(pl.R * pl.n, x, s0, st));
            launches = t1 - t0;
            for (int32_t t = t0; t < t1; ++t) {
                QPA_HIP(launch_dense_tiled_step(pl.n, pl.R, at<float>(ws, pl.o_Jf), bf, s0, s1,
                                                x, m, (t == t1 - 1) ? h : nullptr, t, lam,
                                                a.eta, a.alpha, st));
                std::swap(s0, s1);
            }
            break;
        }
        case Path::DenseMfma: {
            uint32_t *s0 = at<uint32_t>(ws, pl.o_s0), *s1 = at<uint32_t>(ws, pl.o_s1);
            QPA_HIP(launch_mfma_pack_spins(pl.Rp, pl.np, x, s0, st));
            launches = t1 - t0;
            const CanonScalars *sc = at<CanonScalars>(ws, pl.o_sc);
            for (int32_t t = t0; t < t1; ++t) {
                QPA_HIP(launch_mfma_step(pl.Rp, pl.np, at<uint16_t>(ws, pl.o_Jb), bf, sc, s0, s1,
                                         x, m, (t == t1 - 1) ? h : nullptr, t, lam, a.eta,
                                         a.alpha, st));
                std::swap(s0, s1);
            }
            break;
        }
        case Path::Csr: {
            uint64_t *s0 = at<uint64_t>(ws, pl.o_s0), *s1 = at<uint64_t>(ws, pl.o_s1);
            QPA_HIP(launch_csr_pack_spins(pl.n, pl.Rp, pl.G, x, s0, st));
            launches = t1 - t0;
            CsrView c{pl.n, p.row_ptr, p.col, p.weights, p.index_dtype, p.coupling_dtype,
                      pl.is_qubo};
            for (int32_t t = t0; t < t1; ++t) {
                QPA_HIP(launch_csr_step(c, pl.Rp, pl.G, bf, s0, s1, x, m,
                                        (t == t1 - 1) ? h : nullptr, t, lam, a.eta, a.alpha,
                                        pl.is_int, st));
                std::swap(s0, s1);
            }
            break;
        }
    }
    return QPA_OK;
}

qpa_status score(qpa_ctx *ctx, const qpa_problem &p, const Plan &pl, void *ws,
                 const int8_t *spins, double *energy, int64_t *energy_i64, int32_t *best,
                 hipStream_t st) {
    int64_t *ei = energy_i64 ? energy_i64 : at<int64_t>(ws, pl.o_ei);
    QPA_HIP(launch_energy(p, at<int64_t>(ws, pl.o_bi), at<double>(ws, pl.o_bd),
                          at<CanonScalars>(ws, pl.o_sc), spins, pl.R, ei, energy,
                          at<double>(ws, pl.o_part), pl.eblk * pl.R, st));
    if (best) QPA_HIP(launch_argmin(pl.R, pl.is_int ? ei : nullptr, energy, best, st));
    return QPA_OK;
}

qpa_status prologue(qpa_ctx *ctx, const qpa_problem *problem, const qpa_params *params,
                    void *ws, size_t ws_bytes, Plan &pl) {
    if (!ctx) return QPA_E_ARG;
    ctx->err.clear();
    qpa_status s = check_problem(ctx, problem);
    if (s != QPA_OK) return s;
    s = check_params(ctx, params);
    if (s != QPA_OK) return s;
    pl = make_plan(*problem, *params);
    if (!ws) return fail(ctx, QPA_E_ARG, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(ws) % ALIGN) != 0)
        return fail(ctx, QPA_E_ARG, "workspace must be %zu-byte aligned", ALIGN);
    if (ws_bytes < pl.total)
        return fail(ctx, QPA_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes,
                    pl.total);
    QPA_HIP(hipSetDevice(ctx->device));
    return QPA_OK;
}

}  // namespace
}  // namespace qpa

using namespace qpa;

extern "C" {

qpa_status qpa_create(qpa_ctx **out, int device) {
    if (!out) return fail(nullptr, QPA_E_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess)
        return fail(nullptr, QPA_E_DEVICE, "hipGetDeviceCount failed: %s", hipGetErrorString(e));
    if (device < 0 || device >= count)
        return fail(nullptr, QPA_E_DEVICE, "device %d out of range (%d devices)", device, count);
    e = hipSetDevice(device);
    if (e != hipSuccess)
        return fail(nullptr, QPA_E_DEVICE, "hipSetDevice(%d) failed: %s", device,
                    hipGetErrorString(e));
    qpa_ctx *c = new qpa_ctx();
    c->device = device;
    e = hipHostMalloc((void **)&c->host_sc, sizeof(CanonScalars), hipHostMallocDefault);
    if (e != hipSuccess) {
        delete c;
        return fail(nullptr, QPA_E_DEVICE, "hipHostMalloc failed: %s", hipGetErrorString(e));
    }
    *out = c;
    return QPA_OK;
}

void qpa_destroy(qpa_ctx *ctx) {
    if (!ctx) return;
    if (ctx->host_sc) (void)hipHostFree(ctx->host_sc);
    if (ctx->host_lam) (void)hipHostFree(ctx->host_lam);
    for (auto &sp : ctx->spans) {
        (void)hipEventDestroy(sp.a);
        (void)hipEventDestroy(sp.b);
    }
    for (auto ev : ctx->free_events) (void)hipEventDestroy(ev);
    delete ctx;
}

const char *qpa_last_error(const qpa_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_noctx_err.c_str();
}

const char *qpa_status_string(qpa_status s) {
    switch (s) {
        case QPA_OK: return "QPA_OK";
        case QPA_E_ARG: return "QPA_E_ARG";
        case QPA_E_SHAPE: return "QPA_E_SHAPE";
        case QPA_E_ASYM: return "QPA_E_ASYM";
        case QPA_E_RANGE: return "QPA_E_RANGE";
        case QPA_E_WORKSPACE: return "QPA_E_WORKSPACE";
        case QPA_E_DEVICE: return "QPA_E_DEVICE";
        case QPA_E_UNSUPPORTED: return "QPA_E_UNSUPPORTED";
    }
    return "QPA_E_UNKNOWN";
}

const char *qpa_version(void) { return "qpa 0.1 (gfx950)"; }

qpa_status qpa_profile_enable(qpa_ctx *ctx, int32_t enable) {
    if (!ctx) return QPA_E_ARG;
    ctx->prof = enable != 0;
    return QPA_OK;
}

qpa_status qpa_profile_read(qpa_ctx *ctx, double *step_ms, int64_t *step_launches,
                            int32_t reset) {
    if (!ctx || !step_ms || !step_launches) return QPA_E_ARG;
    double total = 0.0;
    int64_t n = 0;
    for (auto &sp : ctx->spans) {
        QPA_HIP(hipEventSynchronize(sp.b));
        float ms = 0.0f;
        QPA_HIP(hipEventElapsedTime(&ms, sp.a, sp.b));
        total += ms;
        n += sp.launches;
    }
    *step_ms = total;
    *step_launches = n;
    if (reset) {
        for (auto &sp : ctx->spans) {
            ctx->free_events.push_back(sp.a);
            ctx->free_events.push_back(sp.b);
        }
        ctx->spans.clear();
    }
    return QPA_OK;
}

qpa_status qpa_workspace_size(qpa_ctx *ctx, const qpa_problem *problem,
                              const qpa_params *params, size_t *bytes) {
    if (!bytes) return fail(ctx, QPA_E_ARG, "bytes is NULL");
    qpa_status s = check_problem(ctx, problem);
    if (s != QPA_OK) return s;
    s = check_params(ctx, params);
    if (s != QPA_OK) return s;
    *bytes = make_plan(*problem, *params).total;
    return QPA_OK;
}

qpa_status qpa_solve(qpa_ctx *ctx, const qpa_problem *problem, const qpa_params *params,
                     void *workspace, size_t workspace_bytes, void *stream,
                     const qpa_outputs *out) {
    Plan pl;
    qpa_status s = prologue(ctx, problem, params, workspace, workspace_bytes, pl);
    if (s != QPA_OK) return s;
    if (!out || !out->energy || !out->best)
        return fail(ctx, QPA_E_ARG, "outputs.energy and outputs.best are required");
    hipStream_t st = static_cast<hipStream_t>(stream);
    void *ws = workspace;
    s = upload_schedule(ctx, *params, at<float>(ws, pl.o_lam), st);
    if (s != QPA_OK) return s;
    s = canonicalise(ctx, *problem, pl, ws, st);
    if (s != QPA_OK) return s;
    int64_t ld_r, ld_i;
    state_strides(pl, ld_r, ld_i);
    float *x = at<float>(ws, pl.o_x), *m = at<float>(ws, pl.o_m);
    QPA_HIP(launch_init_state(pl.n, pl.R, params->seed, params->sigma0, x, m, ld_r, ld_i, pl.Rp,
                              pl.np, st));
    s = run_steps(ctx, *problem, *params, pl, ws, 0, params->steps, false, st);
    if (s != QPA_OK) return s;
    int8_t *spins = out->spins ? out->spins : at<int8_t>(ws, pl.o_sp);
    QPA_HIP(launch_export_spins(pl.n, pl.R, x, ld_r, ld_i, spins, st));
    if (out->x) QPA_HIP(launch_copy_state(pl.n, pl.R, x, ld_r, ld_i, out->x, pl.n, 1, st));
    if (out->m) QPA_HIP(launch_copy_state(pl.n, pl.R, m, ld_r, ld_i, out->m, pl.n, 1, st));
    return score(ctx, *problem, pl, ws, spins, out->energy, out->energy_i64, out->best, st);
}

qpa_status qpa_steps(qpa_ctx *ctx, const qpa_problem *problem, const qpa_params *params,
                     int32_t t0, int32_t t1, float *x_io, float *m_io, float *h_last,
                     void *workspace, size_t workspace_bytes, void *stream) {
    Plan pl;
    qpa_status s = prologue(ctx, problem, params, workspace, workspace_bytes, pl);
    if (s != QPA_OK) return s;
    if (!x_io || !m_io) return fail(ctx, QPA_E_ARG, "x and m are required");
    if (t0 < 0 || t1 < t0 || t1 > params->steps)
        return fail(ctx, QPA_E_ARG, "need 0 <= t0 <= t1 <= steps (got %d, %d, %d)", t0, t1,
                    params->steps);
    hipStream_t st = static_cast<hipStream_t>(stream);
    void *ws = workspace;
    s = upload_schedule(ctx, *params, at<float>(ws, pl.o_lam), st);
    if (s != QPA_OK) return s;
    s = canonicalise(ctx, *problem, pl, ws, st);
    if (s != QPA_OK) return s;
    int64_t ld_r, ld_i;
    state_strides(pl, ld_r, ld_i);
    float *x = at<float>(ws, pl.o_x), *m = at<float>(ws, pl.o_m);
    if (pl.Rp != pl.R || pl.np != pl.n) {
        // padding entries start at zero and stay inert
        QPA_HIP(hipMemsetAsync(x, 0, sizeof(float) * (size_t)(pl.Rp * pl.np), st));
        QPA_HIP(hipMemsetAsync(m, 0, sizeof(float) * (size_t)(pl.Rp * pl.np), st));
    }
    QPA_HIP(launch_copy_state(pl.n, pl.R, x_io, pl.n, 1, x, ld_r, ld_i, st));
    QPA_HIP(launch_copy_state(pl.n, pl.R, m_io, pl.n, 1, m, ld_r, ld_i, st));
    s = run_steps(ctx, *problem, *params, pl, ws, t0, t1, h_last != nullptr, st);
    if (s != QPA_OK) return s;
    QPA_HIP(launch_copy_state(pl.n, pl.R, x, ld_r, ld_i, x_io, pl.n, 1, st));
    QPA_HIP(launch_copy_state(pl.n, pl.R, m, ld_r, ld_i, m_io, pl.n, 1, st));
    if (h_last && t1 > t0)
        QPA_HIP(launch_copy_state(pl.n, pl.R, at<float>(ws, pl.o_h), ld_r, ld_i, h_last, pl.n, 1,
                                  st));
    return QPA_OK;
}

qpa_status qpa_energy(qpa_ctx *ctx, const qpa_problem *problem, const qpa_params *params,
                      const int8_t *spins, double *energy, int64_t *energy_i64,
                      int32_t *best, void *workspace, size_t workspace_bytes, void *stream) {
    Plan pl;
    qpa_status s = prologue(ctx, problem, params, workspace, workspace_bytes, pl);
    if (s != QPA_OK) return s;
    if (!spins || !energy) return fail(ctx, QPA_E_ARG, "spins and energy are required");
    hipStream_t st = static_cast<hipStream_t>(stream);
    s = canonicalise(ctx, *problem, pl, workspace, st);
    if (s != QPA_OK) return s;
    return score(ctx, *problem, pl, workspace, spins, energy, energy_i64, best, st);
}

}  // extern "C"
