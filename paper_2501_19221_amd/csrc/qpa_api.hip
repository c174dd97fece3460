// C ABI of libqpa: argument checks, workspace planning and the order of launches of a
// solve.  Every step of the method runs in the kernels of the other translation units.
#include "qpa_internal.h"

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>

#include <algorithm>
#include <string>
#include <mutex>
#include <thread>
#include <vector>

struct qpa_ctx {
    int device = 0;
    int cus = 256;                          // compute units of the device
    std::string err;
    int32_t *host_flags = nullptr;          // pinned, for device status read-backs
    qpa::CanonScalars *host_sc = nullptr;   // pinned
    float *host_lam = nullptr;              // pinned schedule staging
    size_t host_lam_cap = 0;
    char *host_stage = nullptr;             // pinned, the batch solve's table uploads and
    size_t host_stage_cap = 0;              // read-backs (grown, kept until qpa_destroy)
    void *noalloc_ws = nullptr;             // device address of this device's static workspace
    // step-kernel timing (qpa_profile_*)
    bool prof = false;
    struct Span {
        hipEvent_t a, b;
        int64_t launches;
        int32_t path;
    };
    std::vector<Span> spans;
    std::vector<hipEvent_t> free_events;
    std::vector<int32_t> batch_paths;       // per instance, last qpa_solve_batch
    // step loops captured as HIP graphs (QPA_SOLVE_GRAPH), keyed by every argument the
    // captured launches read; captured on a private stream of default priority
    hipStream_t cap = nullptr;
    struct Graph {
        std::vector<uint8_t> key;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;              // most recently used last
    // sparse kernel choices found by qpa_autotune: shape key -> 0 (streamed kernel) or
    // the resident kernel's replica group
    struct TuneKey {
        int64_t n, nnz;
        int32_t kind, coupling_dtype, index_dtype, replicas;
        bool operator==(const TuneKey &o) const {
            return n == o.n && nnz == o.nnz && kind == o.kind &&
                   coupling_dtype == o.coupling_dtype && index_dtype == o.index_dtype &&
                   replicas == o.replicas;
        }
    };
    std::vector<std::pair<TuneKey, int32_t>> tuned;
    // batch path rates measured by qpa_autotune_batch (0: the built-in estimates):
    // dense tiles in bytes per second (2 bytes per coupling plus 16 per variable and
    // replica, whatever the tile element type), sparse tasks in coupling adds per second
    double batch_dense_Bps = 0.0, batch_sparse_adds = 0.0;
    // streams of default priority for the independent per-instance work of a batch, and
    // the events that order them after and join them back into the caller's stream
    std::vector<hipStream_t> aux;
    std::vector<hipEvent_t> aux_ev;         // [0]: fork, [1 + i]: join of aux[i]
};

namespace qpa {
namespace {

constexpr size_t ALIGN = 256;

inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }
inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

enum class Path { DenseResident, DenseTiled, DenseMfma, Csr, CsrResident, CsrBinned };

int32_t path_code(Path p) {
    switch (p) {
        case Path::DenseResident: return QPA_PATH_DENSE_RESIDENT;
        case Path::DenseTiled: return QPA_PATH_DENSE_TILED;
        case Path::DenseMfma: return QPA_PATH_DENSE_MFMA;
        case Path::CsrResident: return QPA_PATH_CSR_RESIDENT;
        case Path::CsrBinned: return QPA_PATH_CSR_BINNED;
        default: return QPA_PATH_CSR;
    }
}

const char *path_name(Path p) {
    switch (p) {
        case Path::DenseResident: return "dense-resident-fp32";
        case Path::DenseTiled: return "dense-tiled-fp32";
        case Path::DenseMfma: return "dense-mfma-bf16";
        case Path::Csr: return "csr";
        case Path::CsrResident: return "csr-resident";
        case Path::CsrBinned: return "csr-binned";
    }
    return "?";
}

struct Plan {
    Path path;
    int64_t n, R, T;
    int64_t np, Rp;       // padded sizes of the internal state
    int G;                // CSR replica group of the chosen kernel
    int Gs;               // CSR replica group of the streamed kernel (state / spin layout)
    int64_t nwords;       // CSR spin words per group (streamed layout)
    bool is_int, is_qubo;
    bool bin_ok;          // the binned sparse kernels apply (their arrays are allocated)
    BinGeom bg;           // their geometry with one sum per word (the most blocks)
    int64_t eblk;         // energy partial blocks
    // workspace offsets (bytes)
    size_t o_sc, o_cpart, o_lam, o_bf, o_bi, o_bd, o_rabs, o_rmax, o_rk, o_Jf, o_Jb, o_x, o_m, o_h,
        o_s0, o_s1, o_part, o_ei, o_ed, o_sp, o_best, o_words, o_boff, o_bcur, o_btsum,
        o_bsrc, o_bdrec, o_bbits, o_bcrow, total;
};

// Spin words of the streamed layout above which the binned kernels run by default: the
// per-row gather then misses the L2 on nearly every coupling.
constexpr int64_t BIN_AUTO_BYTES = (int64_t)4 << 20;


// batch_rp > 0: state for the batch kernel, [batch_rp/64 groups][n][64].
// cus: compute units of the device (chooses the replica group of the resident sparse
// kernel; the workspace size does not depend on it).
// state = false: no PA state buffers (callers that keep their own, such as SBM).
Plan make_plan(const qpa_problem &p, const qpa_params &a, int64_t batch_rp = 0, int cus = 256,
               bool state = true) {
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
    pl.Gs = 1;
    if (p.format == QPA_FMT_CSR) {
        // one workspace layout for both sparse kernels (the streamed kernel's), so that
        // the choice between them can change without a new workspace
        pl.path = Path::Csr;
        pl.Gs = batch_rp > 0 ? 64 : csr_group_size(pl.R);
        pl.G = pl.Gs;
        pl.Rp = batch_rp > 0 ? batch_rp : round_up(pl.R, pl.Gs);
        pl.nwords = csr_words_per_group(pl.n, pl.Gs);
        if (batch_rp == 0 && cus > 0 && !(a.flags & QPA_SOLVE_STREAMED) &&
            csr_resident_group(pl.n, pl.R, cus) > 0 &&
            csr_resident_lds(pl.n, p.nnz) <= RES_MAX_LDS) {
            pl.path = Path::CsrResident;
            pl.G = csr_resident_group(pl.n, pl.R, cus);
        }
        // binned kernels: int8 / int16 couplings, integer fields, one group of <= 8 lanes
        pl.bin_ok = batch_rp == 0 && cus > 0 && state && pl.is_int &&
                    (p.coupling_dtype == QPA_I8 || p.coupling_dtype == QPA_I16) &&
                    pl.Rp == pl.Gs && pl.Gs <= 8 && bin_geometry(pl.n, pl.Gs, 1, pl.bg);
        if (pl.bin_ok && ((a.flags & QPA_SOLVE_BINNED) ||
                          (!(a.flags & QPA_SOLVE_STREAMED) && pl.path == Path::Csr &&
                           8 * pl.nwords > BIN_AUTO_BYTES))) {
            pl.path = Path::CsrBinned;
            pl.G = pl.Gs;
        }
    } else if (a.precision == QPA_PREC_BF16) {
        pl.path = Path::DenseMfma;
        pl.np = round_up(pl.n, MF_NPAD);
        pl.Rp = round_up(pl.R, MF_BM);
    } else if (dense_resident_fits(pl.n)) {
        pl.path = Path::DenseResident;
    } else {
        pl.path = Path::DenseTiled;
        pl.Rp = dense_fp32_rpad(pl.R);
    }
    pl.eblk = energy_partial_blocks(p);
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
    pl.o_cpart = take(sizeof(double) * 4 * (size_t)CANON_PARTS);
    pl.o_Jf = (pl.path == Path::DenseResident || pl.path == Path::DenseTiled)
                  ? take(sizeof(float) * n * n) : 0;
    pl.o_Jb = pl.path == Path::DenseMfma ? take(sizeof(uint16_t) * np * np) : 0;
    pl.o_x = state ? take(sizeof(float) * Rp * np) : 0;
    pl.o_m = state ? take(sizeof(float) * Rp * np) : 0;
    pl.o_h = state ? take(sizeof(float) * Rp * np) : 0;
    size_t sbytes = 0;
    switch (pl.path) {
        case Path::DenseResident: sbytes = 0; break;
        case Path::DenseTiled: sbytes = sizeof(float) * Rp * n; break;
        case Path::DenseMfma: sbytes = sizeof(uint32_t) * Rp * (np / 8); break;
        case Path::Csr:
        case Path::CsrResident:
        case Path::CsrBinned:
            sbytes = sizeof(uint64_t) * (size_t)(Rp / pl.Gs) * (size_t)pl.nwords;
            break;
    }
    if (!state) sbytes = 0;
    pl.o_s0 = sbytes ? take(sbytes) : 0;
    pl.o_s1 = sbytes ? take(sbytes) : 0;
    pl.o_part = take(sizeof(double) * (size_t)pl.eblk * R);
    pl.o_ei = take(sizeof(int64_t) * R);
    pl.o_ed = take(sizeof(double) * R);
    pl.o_sp = take(sizeof(int8_t) * R * n);
    pl.o_best = take(sizeof(int32_t) * 4);
    pl.o_words = p.format == QPA_FMT_DENSE
                     ? take(sizeof(uint64_t) * R * (size_t)((n + 63) / 64)) : 0;
    if (pl.bin_ok) {
        const size_t nnz = (size_t)std::max<int64_t>(p.nnz, 0), M = (size_t)pl.bg.M;
        pl.o_boff = take(sizeof(int32_t) * (M + 1));
        pl.o_bcur = take(sizeof(int32_t) * M);
        pl.o_btsum = take(sizeof(int32_t) * ((size_t)bin_scan_tiles(pl.bg) + 1));
        pl.o_bsrc = take(sizeof(uint32_t) * nnz);
        pl.o_bdrec = take(sizeof(uint32_t) * nnz);
        pl.o_bbits = take(nnz);
        pl.o_bcrow = take(sizeof(int32_t) * n);
    }
    pl.total = off;
    return pl;
}

// Strides of element (r, i) in the internal state layout of a plan.
void state_strides(const Plan &pl, int64_t &ld_r, int64_t &ld_i) {
    if (pl.path == Path::Csr || pl.path == Path::CsrResident || pl.path == Path::CsrBinned ||
        pl.path == Path::DenseTiled) {
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
    if ((a->flags & ~(QPA_SOLVE_STREAMED | QPA_SOLVE_GRAPH | QPA_SOLVE_BINNED)) != 0)
        return fail(ctx, QPA_E_ARG,
                    "params.flags: only QPA_SOLVE_STREAMED, QPA_SOLVE_BINNED and QPA_SOLVE_GRAPH");
    if ((a->flags & QPA_SOLVE_STREAMED) && (a->flags & QPA_SOLVE_BINNED))
        return fail(ctx, QPA_E_ARG, "QPA_SOLVE_STREAMED and QPA_SOLVE_BINNED exclude each other");
    return QPA_OK;
}

qpa_status check_batch_params(qpa_ctx *ctx, const qpa_params *a) {
    if (!a) return fail(ctx, QPA_E_ARG, "params is NULL");
    qpa_params b = *a;
    const int32_t path = b.flags & ~QPA_SOLVE_GRAPH;
    if (path != 0 && path != QPA_BATCH_SPARSE && path != QPA_BATCH_DENSE)
        return fail(ctx, QPA_E_ARG,
                    "params.flags must be 0, QPA_BATCH_SPARSE or QPA_BATCH_DENSE, optionally "
                    "or-ed with QPA_SOLVE_GRAPH");
    b.flags = 0;
    return check_params(ctx, &b);
}

template <typename T> T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// The context's pinned staging block, at least `bytes` long.  Callers synchronise the
// stream a copy from or into it was issued on before they return, so every call finds it
// idle.
qpa_status host_stage(qpa_ctx *ctx, size_t bytes, char **out) {
    bytes = std::max<size_t>(bytes, 16);
    if (ctx->host_stage_cap < bytes) {
        const size_t cap = std::max(bytes, 2 * ctx->host_stage_cap);
        if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
        ctx->host_stage = nullptr;
        ctx->host_stage_cap = 0;
        QPA_HIP(hipHostMalloc((void **)&ctx->host_stage, cap));
        ctx->host_stage_cap = cap;
    }
    *out = ctx->host_stage;
    return QPA_OK;
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
                                   at<double>(ws, pl.o_rmax), at<double>(ws, pl.o_rk),
                                   at<double>(ws, pl.o_cpart), sc, st));
    } else {
        QPA_HIP(launch_canon_csr(p, bf, at<int64_t>(ws, pl.o_bi), at<double>(ws, pl.o_bd),
                                 at<double>(ws, pl.o_rabs), at<double>(ws, pl.o_rmax),
                                 at<double>(ws, pl.o_rk), at<double>(ws, pl.o_cpart), sc, st));
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
                           hipStream_t st, int64_t &launches, int32_t &ran);

template <typename T> void key_add(std::vector<uint8_t> &k, const T &v) {
    const uint8_t *b = reinterpret_cast<const uint8_t *>(&v);
    k.insert(k.end(), b, b + sizeof(T));
}

constexpr size_t GRAPH_CACHE = 8;

// Launch the step loop `body(stream)` as a HIP graph: captured on the context's private
// stream the first time a key is seen, then replayed on `st`.  The key holds every value
// the captured launches read from the host, so a replay is the same launch sequence.
template <typename F>
qpa_status run_graph(qpa_ctx *ctx, std::vector<uint8_t> key, hipStream_t st, F &&body) {
    for (size_t g = 0; g < ctx->graphs.size(); ++g) {
        if (ctx->graphs[g].key == key) {
            qpa_ctx::Graph hit = ctx->graphs[g];
            ctx->graphs.erase(ctx->graphs.begin() + (std::ptrdiff_t)g);
            ctx->graphs.push_back(hit);
            QPA_HIP(hipGraphLaunch(hit.exec, st));
            return QPA_OK;
        }
    }
    if (!ctx->cap) QPA_HIP(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
    QPA_HIP(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
    qpa_status s = body(ctx->cap);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->cap, &graph);
    if (s != QPA_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    if (e != hipSuccess) return fail(ctx, QPA_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess)
        return fail(ctx, QPA_E_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
    if (ctx->graphs.size() >= GRAPH_CACHE) {
        (void)hipGraphExecDestroy(ctx->graphs.front().exec);
        ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back({std::move(key), exec});
    QPA_HIP(hipGraphLaunch(exec, st));
    return QPA_OK;
}

// Geometry of the binned kernels for this call: as many field sums per LDS word as the
// canonical row bound (sum of |w| plus |b|, read back by canonicalise) allows, hence as few
// blocks as possible.  Never more blocks than the plan's workspace holds.
BinGeom bin_run_geometry(const qpa_ctx *ctx, const Plan &pl) {
    const double bound = ctx->host_sc->max_row;
    const int lanes = (pl.Gs >= 4 && bound < 256.0) ? 4 : (pl.Gs >= 2 && bound < 65536.0) ? 2 : 1;
    BinGeom g;
    if (!bin_geometry(pl.n, pl.Gs, lanes, g)) return pl.bg;
    return g;
}

// Entry order of the binned kernels (once per call, before the step loop).
qpa_status bin_build(qpa_ctx *ctx, const qpa_problem &p, const Plan &pl, void *ws,
                     hipStream_t st) {
    CsrView c{pl.n, p.row_ptr, p.col, p.weights, p.index_dtype, p.coupling_dtype, pl.is_qubo,
              p.nnz};
    QPA_HIP(launch_bin_build(c, bin_run_geometry(ctx, pl), at<int64_t>(ws, pl.o_bi),
                             at<int32_t>(ws, pl.o_boff), at<int32_t>(ws, pl.o_bcur),
                             at<int32_t>(ws, pl.o_btsum), at<uint32_t>(ws, pl.o_bsrc),
                             at<uint32_t>(ws, pl.o_bdrec), at<int32_t>(ws, pl.o_bcrow), st));
    return QPA_OK;
}

bool per_step_path(Path p) {
    return p == Path::DenseTiled || p == Path::DenseMfma || p == Path::Csr ||
           p == Path::CsrBinned;
}

// Run steps t0 .. t1-1 on the internal state of the plan (timed when profiling).
qpa_status run_steps(qpa_ctx *ctx, const qpa_problem &p, const qpa_params &a, const Plan &pl,
                     void *ws, int32_t t0, int32_t t1, bool want_h, hipStream_t st) {
    if (t1 <= t0) return QPA_OK;
    if (pl.path == Path::CsrBinned) {
        qpa_status sb = bin_build(ctx, p, pl, ws, st);
        if (sb != QPA_OK) return sb;
    }
    int64_t launches = 0;
    int32_t ran = path_code(pl.path);
    const bool graph = (a.flags & QPA_SOLVE_GRAPH) && per_step_path(pl.path);
    auto inner = [&](hipStream_t s_) {
        return run_steps_inner(ctx, p, a, pl, ws, t0, t1, want_h, s_, launches, ran);
    };
    auto run = [&]() -> qpa_status {
        if (!graph) return inner(st);
        std::vector<uint8_t> key;
        key_add(key, (int32_t)1);
        key_add(key, p);
        key_add(key, (int32_t)pl.path);
        key_add(key, pl.n);
        key_add(key, pl.R);
        key_add(key, pl.np);
        key_add(key, pl.Rp);
        key_add(key, pl.G);
        key_add(key, pl.total);
        key_add(key, ws);
        key_add(key, a.eta);
        key_add(key, a.alpha);
        key_add(key, a.steps);
        key_add(key, t0);
        key_add(key, t1);
        key_add(key, want_h);
        // the binned kernels' geometry follows the data (row bound), and the entry order
        // built eagerly before the replay must match the captured launches
        key_add(key, pl.path == Path::CsrBinned ? bin_run_geometry(ctx, pl).lanes : 0);
        qpa_status s_ = run_graph(ctx, std::move(key), st, inner);
        launches = t1 - t0;
        return s_;
    };
    if (!ctx->prof) return run();
    qpa_ctx::Span sp{};
    QPA_HIP(take_event(ctx, &sp.a));
    QPA_HIP(take_event(ctx, &sp.b));
    QPA_HIP(hipEventRecord(sp.a, st));
    qpa_status s = run();
    QPA_HIP(hipEventRecord(sp.b, st));
    sp.launches = launches;
    sp.path = ran;
    ctx->spans.push_back(sp);
    return s;
}

qpa_status run_steps_inner(qpa_ctx *ctx, const qpa_problem &p, const qpa_params &a,
                           const Plan &pl, void *ws, int32_t t0, int32_t t1, bool want_h,
                           hipStream_t st, int64_t &launches, int32_t &ran) {
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
            QPA_HIP(launch_sign_f32(pl.Rp * pl.n, x, s0, st));
            launches = t1 - t0;
            for (int32_t t = t0; t < t1; ++t) {
                QPA_HIP(launch_dense_fp32_step(pl.n, pl.Rp, at<float>(ws, pl.o_Jf), bf, s0, s1,
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
            ran = QPA_PATH_DENSE_MFMA;
            const CanonScalars *sc = at<CanonScalars>(ws, pl.o_sc);
            for (int32_t t = t0; t < t1; ++t) {
                QPA_HIP(launch_mfma_step(pl.Rp, pl.np, pl.R, at<uint16_t>(ws, pl.o_Jb), bf, sc,
                                         s0, s1, x, m, (t == t1 - 1) ? h : nullptr, t, lam,
                                         a.eta, a.alpha, st));
                std::swap(s0, s1);
            }
            break;
        }
        case Path::CsrResident: {
            CsrView c{pl.n, p.row_ptr, p.col, p.weights, p.index_dtype, p.coupling_dtype,
                      pl.is_qubo, p.nnz};
            // the canonical row bound (sum of |w| plus |b|, read back by canonicalise)
            // bounds every row's sum of |w|
            const bool small_w = pl.is_int && ctx->host_sc->max_row < 65536.0;
            QPA_HIP(launch_csr_resident(c, pl.G, pl.R, pl.Rp, pl.is_int, small_w, bf, x, m, h, t0,
                                        t1, lam, a.eta, a.alpha, st));
            launches = 1;
            break;
        }
        case Path::CsrBinned: {
            uint64_t *s0 = at<uint64_t>(ws, pl.o_s0), *s1 = at<uint64_t>(ws, pl.o_s1);
            QPA_HIP(launch_csr_pack_spins(pl.n, pl.Rp, pl.Gs, x, s0, st));
            const int32_t *off = at<int32_t>(ws, pl.o_boff);
            const uint32_t *src = at<uint32_t>(ws, pl.o_bsrc), *drec = at<uint32_t>(ws, pl.o_bdrec);
            const BinGeom g = bin_run_geometry(ctx, pl);
            launches = 2 * (int64_t)(t1 - t0);
            for (int32_t t = t0; t < t1; ++t) {
                QPA_HIP(launch_bin_step(g, pl.n, pl.nwords, off, src, drec,
                                        at<uint8_t>(ws, pl.o_bbits), at<int32_t>(ws, pl.o_bcrow),
                                        s0, s1, x, m, (t == t1 - 1) ? h : nullptr, t, lam, a.eta,
                                        a.alpha, ctx->cus, st));
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
                          at<double>(ws, pl.o_part), pl.eblk * pl.R,
                          pl.o_words ? at<uint64_t>(ws, pl.o_words) : nullptr, st));
    if (best) QPA_HIP(launch_argmin(pl.R, pl.is_int ? ei : nullptr, energy, best, st));
    return QPA_OK;
}

// Key of a sparse instance's shape for the tuned-choice table (no allocation: the
// allocation-free solve looks it up too).
qpa_ctx::TuneKey tune_key(const qpa_problem &p, const qpa_params &a) {
    return qpa_ctx::TuneKey{p.n, p.nnz, p.kind, p.coupling_dtype, p.index_dtype, a.replicas};
}

constexpr int32_t TUNE_BINNED = QPA_TUNE_BINNED;

bool resident_ok(const qpa_problem &p, int G) {
    if (p.n > RES_MAX_N || csr_resident_lds(p.n, p.nnz) > RES_MAX_LDS) return false;
    const int64_t v = (p.n + 1023) / 1024;
    const int64_t vp = v <= 1 ? 1 : v <= 2 ? 2 : v <= 4 ? 4 : 8;
    return v <= 8 && vp * G <= 16;
}

// Use the kernel qpa_autotune chose for this shape (unless the caller forced the
// streamed kernel).  Both sparse kernels share the workspace layout.
void apply_tuning(qpa_ctx *ctx, const qpa_problem &p, const qpa_params &a, Plan &pl) {
    if (p.format != QPA_FMT_CSR || (a.flags & (QPA_SOLVE_STREAMED | QPA_SOLVE_BINNED)) ||
        ctx->tuned.empty())
        return;
    const qpa_ctx::TuneKey k = tune_key(p, a);
    for (const auto &e : ctx->tuned) {
        if (!(e.first == k)) continue;
        if (e.second == 0) {
            pl.path = Path::Csr;
            pl.G = pl.Gs;
        } else if (e.second == TUNE_BINNED) {
            if (pl.bin_ok) {
                pl.path = Path::CsrBinned;
                pl.G = pl.Gs;
            }
        } else if (resident_ok(p, e.second)) {
            pl.path = Path::CsrResident;
            pl.G = e.second;
        }
        return;
    }
}

qpa_status prologue(qpa_ctx *ctx, const qpa_problem *problem, const qpa_params *params,
                    void *ws, size_t ws_bytes, Plan &pl) {
    if (!ctx) return QPA_E_ARG;
    ctx->err.clear();
    qpa_status s = check_problem(ctx, problem);
    if (s != QPA_OK) return s;
    s = check_params(ctx, params);
    if (s != QPA_OK) return s;
    pl = make_plan(*problem, *params, 0, ctx->cus);
    apply_tuning(ctx, *problem, *params, pl);
    if ((params->flags & QPA_SOLVE_BINNED) && pl.path != Path::CsrBinned)
        return fail(ctx, QPA_E_UNSUPPORTED,
                    "QPA_SOLVE_BINNED needs a CSR problem with int8 or int16 couplings, "
                    "integer fields and at most 8 replicas");
    if (!ws) return fail(ctx, QPA_E_ARG, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(ws) % ALIGN) != 0)
        return fail(ctx, QPA_E_ARG, "workspace must be %zu-byte aligned", ALIGN);
    if (ws_bytes < pl.total)
        return fail(ctx, QPA_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes,
                    pl.total);
    QPA_HIP(hipSetDevice(ctx->device));
    return QPA_OK;
}

// Relaxed-gradient workspace of a batch (a single instance is a batch of one): each
// instance's FP32 canonical buffers (no PA state), the instance tables, then the stacked
// state vectors [rows][Rp], the checkpoints, the stored states of a segment, the reverse
// vectors and the per-step partial tables.
struct RelPlan {
    std::vector<Plan> inst;
    std::vector<size_t> base;
    std::vector<int64_t> row0;
    int64_t rows = 0, Rp = 0;
    int64_t blocks_all = 0;        // blocks of 64 rows over every instance
    int32_t C = 0;                 // 64-replica chunks of a row
    int32_t k = 1, nseg = 0;
    // partial slots of a step: the element-wise pass over all rows writes slots
    // [0, nblk_all); a gather step writes each CSR group's blocks and then each dense
    // instance's tiles, [0, nblk_gather); nblk = the larger of the two
    int32_t nblk = 0, nblk_all = 0, nblk_gather = 0;
    struct Group {
        int32_t wdt, idt, first, count, slot0;
        int64_t items, blocks;     // rows, and blocks of 64 rows (the gather's work items)
    };
    std::vector<Group> groups;     // CSR instances by (coupling, index) type
    std::vector<int32_t> csr_order;   // instance indices, grouped
    std::vector<int32_t> dense_slot;  // per instance: first tile slot (-1 for CSR)
    size_t o_tab_all = 0, o_tab_csr = 0, o_lam = 0, o_x0 = 0, o_x1 = 0, o_m = 0, o_ckpt = 0,
           o_seg = 0, o_xbar = 0, o_yb = 0, o_mu0 = 0, o_mu1 = 0, o_part = 0, o_ploss = 0,
           total = 0;
    size_t vec_bytes() const { return sizeof(float) * (size_t)rows * (size_t)Rp; }
};

qpa_status make_rel_plan(qpa_ctx *ctx, int32_t count, const qpa_problem *probs,
                         const qpa_params &a, int32_t k, RelPlan &rp) {
    if (k < 1) return fail(ctx, QPA_E_ARG, "ckpt_every must be >= 1");
    if (count < 1) return fail(ctx, QPA_E_ARG, "count must be >= 1");
    if (!probs) return fail(ctx, QPA_E_ARG, "problems is NULL");
    qpa_params a32 = a;
    a32.precision = QPA_PREC_FP32;
    a32.flags = 0;
    rp.inst.assign(count, Plan{});
    rp.base.assign(count, 0);
    rp.row0.assign(count, 0);
    rp.dense_slot.assign(count, -1);
    rp.groups.clear();
    rp.csr_order.clear();
    rp.rows = 0;
    bool any_dense = false;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes);
        return o;
    };
    for (int32_t q = 0; q < count; ++q) {
        qpa_status s = check_problem(ctx, &probs[q]);
        if (s != QPA_OK) {
            std::string msg = "instance " + std::to_string(q) + ": " + ctx->err;
            return fail(ctx, s, "%s", msg.c_str());
        }
        // FP32 couplings: a dense instance gets its canonical FP32 matrix
        const Plan pl = make_plan(probs[q], a32, 0, 256, false);
        rp.inst[q] = pl;
        rp.base[q] = take(pl.total);
        rp.row0[q] = rp.rows;
        rp.rows += probs[q].n;
        any_dense = any_dense || probs[q].format == QPA_FMT_DENSE;
    }
    rp.Rp = round_up(a.replicas, any_dense ? 128 : 64);
    rp.C = (int32_t)(rp.Rp / 64);
    rp.k = k;
    rp.nseg = (int32_t)((a.steps + k - 1) / k);
    // CSR instances grouped by (coupling, index) type, in index order within a group
    for (int32_t q = 0; q < count; ++q) {
        if (probs[q].format != QPA_FMT_CSR) continue;
        const int32_t wdt = probs[q].coupling_dtype, idt = probs[q].index_dtype;
        bool found = false;
        for (auto &g : rp.groups) found = found || (g.wdt == wdt && g.idt == idt);
        if (!found) rp.groups.push_back({wdt, idt, 0, 0, 0, 0, 0});
    }
    int32_t slot = 0;
    for (auto &g : rp.groups) {
        g.first = (int32_t)rp.csr_order.size();
        for (int32_t q = 0; q < count; ++q)
            if (probs[q].format == QPA_FMT_CSR && probs[q].coupling_dtype == g.wdt &&
                probs[q].index_dtype == g.idt) {
                rp.csr_order.push_back(q);
                g.items += probs[q].n;
                g.blocks += (probs[q].n + 63) / 64;
            }
        g.count = (int32_t)rp.csr_order.size() - g.first;
        g.slot0 = slot;
        slot += (int32_t)rel_gather_blocks(g.blocks, rp.C);
    }
    for (int32_t q = 0; q < count; ++q) {
        if (probs[q].format != QPA_FMT_DENSE) continue;
        rp.dense_slot[q] = slot;
        slot += (int32_t)rel_tile_blocks(probs[q].n, rp.Rp);
    }
    rp.nblk_gather = slot;
    rp.blocks_all = 0;
    for (int32_t q = 0; q < count; ++q) rp.blocks_all += (probs[q].n + 63) / 64;
    rp.nblk_all = (int32_t)rel_gather_blocks(rp.blocks_all, rp.C);
    rp.nblk = std::max(rp.nblk_gather, rp.nblk_all);
    const size_t V = rp.vec_bytes();
    rp.o_tab_all = take(sizeof(RelInst) * (size_t)count);
    rp.o_tab_csr = take(sizeof(RelInst) * std::max<size_t>(rp.csr_order.size(), 1));
    rp.o_lam = take(sizeof(float) * (size_t)std::max<int32_t>(a.steps, 1));
    rp.o_x0 = take(V);
    rp.o_x1 = take(V);
    rp.o_m = take(V);
    rp.o_ckpt = take(V * 2 * (size_t)std::max(rp.nseg, 1));
    rp.o_seg = take(V * 3 * (size_t)(std::min(k, std::max(a.steps, 1)) + 1));
    rp.o_xbar = take(V);
    rp.o_yb = take(V);
    rp.o_mu0 = take(V);
    rp.o_mu1 = take(V);
    rp.o_part = take(sizeof(double) * 3 * (size_t)rp.nblk * (size_t)std::max(a.steps, 1));
    rp.o_ploss = take(sizeof(double) * (size_t)rp.nblk);
    rp.total = off;
    return QPA_OK;
}

constexpr int64_t BATCH_MAX_N = 4096;
static_assert(BATCH_MAX_N <= EBITS_MAX_N, "every densified batch instance fits the batched energies");

// Dense matrix-core buffers of a batch instance that may run as BF16 tiles.
struct DenseSlot {
    bool cand = false;
    int64_t np = 0, Rp = 0;
    size_t o_Jb = 0, o_bfp = 0, o_x = 0, o_m = 0, o_s0 = 0, o_s1 = 0;
};

struct BatchPlan {
    std::vector<Plan> inst;          // per-instance single-solve plans (canonical buffers)
    std::vector<size_t> base;        // byte offset of each instance's region
    std::vector<DenseSlot> dense;
    size_t o_tasks, o_tiles, o_score, o_scall, o_slot, o_canon, o_counter, o_lam, o_i8s_tab,
        o_i8s_stats, total;
    int32_t ntasks, ntiles_max, max_n;
    int32_t inst_tiles_max;   // most tiles of one dense candidate
};

// Workgroup i of a launch runs on compute die (XCD) i mod XCDS, each with its own L2.
constexpr int32_t XCDS = 8;

// Lay a tile list (tiles of one instance consecutive) out so that every instance's tiles
// run on one compute die: instances go, in list order, to the die with the fewest tiles so
// far, and entry XCDS * s + d of the table is die d's s-th tile; shorter dies are filled
// with np = 0 entries, which the kernel skips.  The tiles of an instance then share that
// die's L2 copy of its spins, which each tile reads whole.
std::vector<MfmaTile> by_compute_die(const std::vector<MfmaTile> &in) {
    std::vector<std::vector<MfmaTile>> q(XCDS);
    std::vector<size_t> load(XCDS, 0);
    for (size_t a = 0; a < in.size();) {
        size_t b = a + 1;
        while (b < in.size() && in[b].s0 == in[a].s0) ++b;
        const size_t d = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
        q[d].insert(q[d].end(), in.begin() + (std::ptrdiff_t)a, in.begin() + (std::ptrdiff_t)b);
        load[d] += b - a;
        a = b;
    }
    const size_t L = *std::max_element(load.begin(), load.end());
    std::vector<MfmaTile> out(XCDS * L, MfmaTile{});
    for (size_t d = 0; d < (size_t)XCDS; ++d)
        for (size_t s = 0; s < q[d].size(); ++s) out[XCDS * s + d] = q[d][s];
    return out;
}

// Cost model of one PA step of one instance on the two batch paths, in seconds: work
// over a rate.  The rates are the context's, measured by qpa_autotune_batch on this
// device for the caller's instances; before any measurement, estimates from earlier
// measurements on MI355X (the sparse task kernel about 1e12 signed coupling adds per
// second, the grouped matrix-core step about 3e12 bytes per second).  The grouped step's
// work is its memory traffic: the couplings (2 bytes per element in BF16, or 4 bytes per
// stored entry for integer couplings sparse enough for entry lists: at most a tenth of
// the padded matrix is assumed here, the exact test runs on the device) and x, m.
constexpr double SPARSE_ADDS_DEFAULT = 1.0e12, DENSE_BPS_DEFAULT = 3.0e12;
double csr_step_work(int64_t nnz, int64_t R) { return (double)nnz * (double)R; }
double dense_step_work(int64_t np, int64_t R, int64_t nnz = -1) {
    const double J = nnz >= 0 ? 4.0 * (double)nnz : (double)np * (double)np * 2.0;
    return J + 16.0 * (double)R * (double)np;
}
bool likely_sparse_i8(const qpa_problem &p, int64_t np) {
    return dtype_is_int(p.coupling_dtype) && (double)p.nnz <= 0.1 * (double)np * (double)np;
}
double csr_step_cost(const qpa_ctx *ctx, int64_t nnz, int64_t R) {
    const double r = ctx && ctx->batch_sparse_adds > 0.0 ? ctx->batch_sparse_adds
                                                        : SPARSE_ADDS_DEFAULT;
    return csr_step_work(nnz, R) / r;
}
double dense_step_cost(const qpa_ctx *ctx, int64_t np, int64_t R, int64_t nnz = -1) {
    const double r = ctx && ctx->batch_dense_Bps > 0.0 ? ctx->batch_dense_Bps : DENSE_BPS_DEFAULT;
    return dense_step_work(np, R, nnz) / r;
}

// Per instance: the canonical buffers, energy scratch and [groups][n][64] state of a CSR
// plan, laid out one after the other; then the task table, the queue counter and the
// shared schedule.
qpa_status make_batch_plan(qpa_ctx *ctx, int32_t count, const qpa_problem *probs,
                           const qpa_params &a, BatchPlan &bp) {
    if (count < 1) return fail(ctx, QPA_E_ARG, "count must be >= 1");
    if (!probs) return fail(ctx, QPA_E_ARG, "problems is NULL");
    bp.inst.resize(count);
    bp.base.resize(count);
    bp.dense.clear();
    size_t off = 0;
    bp.ntasks = 0;
    bp.ntiles_max = 0;
    bp.inst_tiles_max = 0;
    bp.max_n = 0;
    const int64_t groups = (a.replicas + 63) / 64;
    for (int32_t k = 0; k < count; ++k) {
        qpa_status s = check_problem(ctx, &probs[k]);
        if (s != QPA_OK) {
            std::string msg = "instance " + std::to_string(k) + ": " + ctx->err;
            return fail(ctx, s, "%s", msg.c_str());
        }
        if (probs[k].format != QPA_FMT_CSR)
            return fail(ctx, QPA_E_UNSUPPORTED, "instance %d: batches take CSR problems", k);
        if (probs[k].n > BATCH_MAX_N)
            return fail(ctx, QPA_E_UNSUPPORTED, "instance %d: n=%lld exceeds the batch limit %lld",
                        k, (long long)probs[k].n, (long long)BATCH_MAX_N);
        Plan pl = make_plan(probs[k], a, groups * 64);
        bp.base[k] = off;
        off += align_up(pl.total);
        bp.inst[k] = pl;
        bp.ntasks += (int32_t)groups;
        bp.max_n = std::max<int32_t>(bp.max_n, (int32_t)probs[k].n);
        // dense BF16 candidate: exact couplings (integer weights, checked <= 256 on the
        // device) or BF16 requested, and cheaper by the cost model
        DenseSlot ds;
        const bool exact_ok = pl.is_int || a.precision == QPA_PREC_BF16;
        // np a multiple of the int8 tiles' 256 variables (BF16 tiles take 128)
        const int64_t np = round_up(probs[k].n, MF_BN8), Rp = round_up(a.replicas, MF_BM);
        const bool cheaper =
            dense_step_cost(ctx, np, a.replicas, likely_sparse_i8(probs[k], np) ? probs[k].nnz : -1) <
            csr_step_cost(ctx, probs[k].nnz, a.replicas);
        const int32_t force = a.flags & (QPA_BATCH_SPARSE | QPA_BATCH_DENSE);
        if (exact_ok && force != QPA_BATCH_SPARSE && (cheaper || force == QPA_BATCH_DENSE)) {
            ds.cand = true;
            ds.np = np;
            ds.Rp = Rp;
            auto tk = [&](size_t bytes) {
                size_t o = off;
                off += align_up(bytes);
                return o;
            };
            ds.o_Jb = tk(sizeof(uint16_t) * (size_t)(np * np));
            ds.o_bfp = tk(sizeof(float) * (size_t)np);
            ds.o_x = tk(sizeof(float) * (size_t)(Rp * np));
            ds.o_m = tk(sizeof(float) * (size_t)(Rp * np));
            // room for byte spins (int8 tiles), twice the pair words of BF16 tiles
            ds.o_s0 = tk((size_t)(Rp * np));
            ds.o_s1 = tk((size_t)(Rp * np));
            const int32_t it = (int32_t)((np / MF_BN) * (Rp / MF_BM));
            bp.ntiles_max += it;
            bp.inst_tiles_max = std::max(bp.inst_tiles_max, it);
        }
        bp.dense.push_back(ds);
    }
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes);
        return o;
    };
    bp.o_tasks = take(sizeof(BatchTask) * (size_t)bp.ntasks);
    // each of the three tile lists (BF16, int8, sparse int8) may gain up to
    // XCDS * inst_tiles_max filler entries when it is laid out by compute die
    bp.o_tiles = take(sizeof(MfmaTile) *
                      (size_t)std::max(bp.ntiles_max + 3 * XCDS * bp.inst_tiles_max, 1));
    bp.o_score = take(sizeof(ScoreTask) * (size_t)std::max(count, 1));
    bp.o_scall = take(sizeof(CanonScalars) * (size_t)std::max(count, 1));
    bp.o_slot = take(sizeof(SlotInitTask) * (size_t)std::max(count, 1));
    bp.o_canon = take(sizeof(CanonTask) * (size_t)std::max(count, 1));
    bp.o_counter = take(sizeof(int32_t));
    bp.o_lam = take(sizeof(float) * (size_t)std::max<int32_t>(a.steps, 1));
    bp.o_i8s_tab = take(sizeof(I8sTask) * (size_t)std::max(count, 1));
    bp.o_i8s_stats = take(2 * sizeof(int32_t) * (size_t)std::max(count, 1));
    bp.total = off;
    return QPA_OK;
}

// SBM workspace: the FP32 plan's canonical and scoring buffers (no PA state), then the
// double-buffered positions, momenta, fields, c0 and the power method's vectors.
struct SbmPlan {
    Plan base;
    int64_t Rp, pblk;
    int Gres;                 // replicas per workgroup of the resident sparse kernel, 0: none
    size_t o_q0, o_q1, o_p, o_g, o_c0, o_pv, o_pw, o_pp, o_nrm, o_atab, total;
};

qpa_status check_sbm_params(qpa_ctx *ctx, const qpa_sbm_params *s) {
    if (!s) return fail(ctx, QPA_E_ARG, "params is NULL");
    if (s->replicas < 1) return fail(ctx, QPA_E_ARG, "replicas must be >= 1");
    if (s->steps < 0) return fail(ctx, QPA_E_ARG, "steps must be >= 0");
    if (!(s->a0 > 0.0f) || !std::isfinite(s->a0)) return fail(ctx, QPA_E_ARG, "a0 must be > 0");
    if (!(s->dt > 0.0f) || !std::isfinite(s->dt)) return fail(ctx, QPA_E_ARG, "dt must be > 0");
    if (!(s->c0 >= 0.0f) || !std::isfinite(s->c0))
        return fail(ctx, QPA_E_ARG, "c0 must be >= 0 (0: from the power method)");
    if (!std::isfinite(s->sigma0)) return fail(ctx, QPA_E_ARG, "sigma0 must be finite");
    if (s->power_iters < 0) return fail(ctx, QPA_E_ARG, "power_iters must be >= 0");
    if ((s->flags & ~(QPA_SOLVE_GRAPH | QPA_SOLVE_STREAMED)) != 0)
        return fail(ctx, QPA_E_ARG, "params.flags: only QPA_SOLVE_STREAMED and QPA_SOLVE_GRAPH");
    return QPA_OK;
}

SbmPlan make_sbm_plan(const qpa_problem &p, const qpa_sbm_params &s, int cus = 256) {
    qpa_params a{};
    a.replicas = s.replicas;
    a.steps = 0;
    a.precision = QPA_PREC_FP32;
    a.flags = QPA_SOLVE_STREAMED;
    SbmPlan sp;
    sp.base = make_plan(p, a, 0, 0, false);
    sp.Rp = sbm_rpad(p, s.replicas);
    sp.pblk = pw_blocks(p);
    sp.Gres = (s.flags & QPA_SOLVE_STREAMED) ? 0 : sbm_resident_group(p, s.replicas, cus);
    size_t off = sp.base.total;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes);
        return o;
    };
    const size_t RN = (size_t)sp.Rp * (size_t)p.n;
    sp.o_q0 = take(sizeof(float) * RN);
    sp.o_q1 = take(sizeof(float) * RN);
    sp.o_p = take(sizeof(float) * RN);
    sp.o_g = take(sizeof(float) * RN);
    sp.o_c0 = take(sizeof(float));
    sp.o_pv = take(sizeof(double) * (size_t)p.n);
    sp.o_pw = take(sizeof(double) * (size_t)p.n);
    sp.o_pp = take(sizeof(double) * (size_t)sp.pblk);
    sp.o_nrm = take(sizeof(double) * 2);
    sp.o_atab = take(sizeof(float) * (size_t)std::max<int32_t>(s.steps, 1));
    sp.total = off;
    return sp;
}

}  // namespace
}  // namespace qpa

using namespace qpa;

// ---------------------------------------------------------------- static workspace
// Workspace of qpa_solve_noalloc: a file-scope device array, one copy per device.  In
// host code its name is only a host-side stand-in, never a device address: the address
// is looked up once per device (with that device current) and kept in the table below;
// kernels and copies get that address only.
static __device__ __align__(256) unsigned char scratch[QPA_NOALLOC_WORKSPACE_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of `device`'s copy of the static workspace; `device` must be current.
hipError_t scratch_address(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr || (reinterpret_cast<uintptr_t>(ptr) % ALIGN) != 0) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace

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
    (void)hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device);
    if (c->cus < 1) c->cus = 1;
    e = hipHostMalloc((void **)&c->host_sc, sizeof(CanonScalars), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&c->host_flags, sizeof(int32_t) * 4, hipHostMallocDefault);
    // the schedule staging buffer, sized for every allocation-free solve
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&c->host_lam, sizeof(float) * (size_t)QPA_NOALLOC_MAX_STEPS,
                          hipHostMallocDefault);
    if (e == hipSuccess) c->host_lam_cap = (size_t)QPA_NOALLOC_MAX_STEPS;
    if (e != hipSuccess) {
        if (c->host_sc) (void)hipHostFree(c->host_sc);
        if (c->host_flags) (void)hipHostFree(c->host_flags);
        delete c;
        return fail(nullptr, QPA_E_DEVICE, "hipHostMalloc failed: %s", hipGetErrorString(e));
    }
    e = scratch_address(device, &c->noalloc_ws);
    if (e != hipSuccess) {
        (void)hipHostFree(c->host_sc);
        (void)hipHostFree(c->host_flags);
        (void)hipHostFree(c->host_lam);
        delete c;
        return fail(nullptr, QPA_E_DEVICE, "static workspace of device %d: %s", device,
                    hipGetErrorString(e));
    }
    *out = c;
    return QPA_OK;
}

void qpa_destroy(qpa_ctx *ctx) {
    if (!ctx) return;
    for (auto &g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    if (ctx->host_sc) (void)hipHostFree(ctx->host_sc);
    if (ctx->host_flags) (void)hipHostFree(ctx->host_flags);
    if (ctx->host_lam) (void)hipHostFree(ctx->host_lam);
    if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
    for (auto &sp : ctx->spans) {
        (void)hipEventDestroy(sp.a);
        (void)hipEventDestroy(sp.b);
    }
    for (auto ev : ctx->free_events) (void)hipEventDestroy(ev);
    for (auto a : ctx->aux) (void)hipStreamDestroy(a);
    for (auto ev : ctx->aux_ev) (void)hipEventDestroy(ev);
    delete ctx;
}

const char *qpa_last_error(const qpa_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_noctx_err.c_str();
}

const char *qpa_status_string(qpa_status s) {
    // a C caller may pass any int: read the bits as an int, not as the enumeration
    int v = 0;
    memcpy(&v, &s, sizeof(v));
    switch (v) {
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
    return qpa_profile_read_path(ctx, QPA_PATH_ALL, step_ms, step_launches, reset);
}

qpa_status qpa_batch_paths(const qpa_ctx *ctx, int32_t count, int32_t *paths) {
    if (!ctx || !paths) return QPA_E_ARG;
    if (count != (int32_t)ctx->batch_paths.size()) return QPA_E_ARG;
    std::copy(ctx->batch_paths.begin(), ctx->batch_paths.end(), paths);
    return QPA_OK;
}

qpa_status qpa_profile_read_path(qpa_ctx *ctx, int32_t path, double *step_ms,
                                 int64_t *step_launches, int32_t reset) {
    if (!ctx || !step_ms || !step_launches) return QPA_E_ARG;
    if (path < QPA_PATH_ALL || path > QPA_PATH_CSR_BINNED)
        return fail(ctx, QPA_E_ARG, "unknown path %d", path);
    double total = 0.0;
    int64_t n = 0;
    for (auto &sp : ctx->spans) {
        if (path != QPA_PATH_ALL && sp.path != path) continue;
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

qpa_status qpa_solve_track(qpa_ctx *ctx, const qpa_problem *problem,
                           const qpa_params *params, int32_t every, void *workspace,
                           size_t workspace_bytes, void *stream, const qpa_outputs *out,
                           const qpa_track_outputs *track) {
    Plan pl;
    qpa_status s = prologue(ctx, problem, params, workspace, workspace_bytes, pl);
    if (s != QPA_OK) return s;
    if (!out || !out->energy || !out->best)
        return fail(ctx, QPA_E_ARG, "outputs.energy and outputs.best are required");
    if (!track || !track->best_energy || !track->best_step || !track->best_spins)
        return fail(ctx, QPA_E_ARG,
                    "track.best_energy, track.best_step and track.best_spins are required");
    if (every < 1) return fail(ctx, QPA_E_ARG, "every must be >= 1 (got %d)", every);
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
    int8_t *spins = out->spins ? out->spins : at<int8_t>(ws, pl.o_sp);
    // segments of `every` steps (a split run gives the bits of an uninterrupted one); the
    // state after each is scored like the final one and offered to the track
    const int32_t T = params->steps;
    int32_t t0 = 0;
    bool first = true;
    do {
        const int32_t t1 = (int32_t)std::min<int64_t>((int64_t)t0 + every, T);
        if (t1 > t0) {
            s = run_steps(ctx, *problem, *params, pl, ws, t0, t1, false, st);
            if (s != QPA_OK) return s;
        }
        QPA_HIP(launch_export_spins(pl.n, pl.R, x, ld_r, ld_i, spins, st));
        s = score(ctx, *problem, pl, ws, spins, out->energy, out->energy_i64,
                  t1 == T ? out->best : nullptr, st);
        if (s != QPA_OK) return s;
        QPA_HIP(launch_track_best(pl.n, pl.R, out->energy, spins, t1, first, track->best_energy,
                                  track->best_step, track->best_spins, st));
        first = false;
        t0 = t1;
    } while (t0 < T);
    if (out->x) QPA_HIP(launch_copy_state(pl.n, pl.R, x, ld_r, ld_i, out->x, pl.n, 1, st));
    if (out->m) QPA_HIP(launch_copy_state(pl.n, pl.R, m, ld_r, ld_i, out->m, pl.n, 1, st));
    return QPA_OK;
}

qpa_status qpa_solve_noalloc(qpa_ctx *ctx, const qpa_problem *problem, const qpa_params *params,
                             void *stream, const qpa_outputs *out) {
    if (!ctx) return QPA_E_ARG;
    ctx->err.clear();
    if (!ctx->noalloc_ws) return fail(ctx, QPA_E_DEVICE, "no static workspace on this device");
    if (!params) return fail(ctx, QPA_E_ARG, "params is NULL");
    if (params->flags & QPA_SOLVE_GRAPH)
        return fail(ctx, QPA_E_UNSUPPORTED,
                    "QPA_SOLVE_GRAPH captures a graph, which allocates; not taken here");
    if (params->steps > QPA_NOALLOC_MAX_STEPS)
        return fail(ctx, QPA_E_UNSUPPORTED, "steps = %d exceeds QPA_NOALLOC_MAX_STEPS = %d",
                    params->steps, QPA_NOALLOC_MAX_STEPS);
    size_t need = 0;
    qpa_status s = qpa_workspace_size(ctx, problem, params, &need);
    if (s != QPA_OK) return s;
    if (need > QPA_NOALLOC_WORKSPACE_BYTES)
        return fail(ctx, QPA_E_WORKSPACE,
                    "the problem needs %zu bytes of workspace; the static workspace holds %zu",
                    need, (size_t)QPA_NOALLOC_WORKSPACE_BYTES);
    // the staging buffer reserved by qpa_create holds the schedule (no hipHostMalloc);
    // profiling spans would create events, so none are recorded
    const bool prof = ctx->prof;
    ctx->prof = false;
    s = qpa_solve(ctx, problem, params, ctx->noalloc_ws, QPA_NOALLOC_WORKSPACE_BYTES, stream,
                  out);
    ctx->prof = prof;
    return s;
}

}  // extern "C"

namespace qpa {
namespace {

// The relaxed forward pass, and with gradients the checkpointed reverse pass, of a batch.
qpa_status relaxed_run(qpa_ctx *ctx, int32_t count, const qpa_problem *probs,
                       const qpa_params *params, int32_t k, double scale, void *ws,
                       size_t ws_bytes, hipStream_t st, double *loss, double *d_eta,
                       double *d_alpha, double *d_lambda) {
    if (!ctx) return QPA_E_ARG;
    ctx->err.clear();
    qpa_status s = check_params(ctx, params);
    if (s != QPA_OK) return s;
    if (!loss) return fail(ctx, QPA_E_ARG, "loss is required");
    const bool grads = d_eta || d_alpha || d_lambda;
    if (grads && (!d_eta || !d_alpha || (params->steps > 0 && !d_lambda)))
        return fail(ctx, QPA_E_ARG,
                    "d_eta, d_alpha and d_lambda are all required (or all NULL: loss only)");
    if (!std::isfinite(scale)) return fail(ctx, QPA_E_ARG, "scale must be finite");
    RelPlan rp;
    s = make_rel_plan(ctx, count, probs, *params, k, rp);
    if (s != QPA_OK) return s;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % ALIGN) != 0)
        return fail(ctx, QPA_E_ARG, "workspace must be non-NULL and %zu-byte aligned", ALIGN);
    if (ws_bytes < rp.total)
        return fail(ctx, QPA_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes,
                    rp.total);
    QPA_HIP(hipSetDevice(ctx->device));
    float *lam = at<float>(ws, rp.o_lam);
    s = upload_schedule(ctx, *params, lam, st);
    if (s != QPA_OK) return s;
    for (int32_t q = 0; q < count; ++q) {
        s = canonicalise(ctx, probs[q], rp.inst[q], at<char>(ws, rp.base[q]), st);
        if (s != QPA_OK) {
            std::string msg = "instance " + std::to_string(q) + ": " + ctx->err;
            return fail(ctx, s, "%s", msg.c_str());
        }
    }
    // instance tables: every instance (element-wise pass) and the CSR ones by group
    auto inst_entry = [&](int32_t q, int64_t item0, int64_t blk0) {
        const qpa_problem &p = probs[q];
        RelInst e{};
        if (p.format == QPA_FMT_CSR) {
            e.rp = p.row_ptr;
            e.col = p.col;
            e.w = p.weights;
        }
        e.b = at<float>(at<char>(ws, rp.base[q]), rp.inst[q].o_bf);
        e.n = p.n;
        e.row0 = rp.row0[q];
        e.item0 = item0;
        e.blk0 = blk0;
        e.skip_diag = p.kind == QPA_KIND_QUBO ? 1 : 0;
        return e;
    };
    std::vector<RelInst> tab_all(count), tab_csr(std::max<size_t>(rp.csr_order.size(), 1));
    int64_t blk_all = 0;
    for (int32_t q = 0; q < count; ++q) {
        tab_all[q] = inst_entry(q, rp.row0[q], blk_all);
        blk_all += (probs[q].n + 63) / 64;
    }
    for (const auto &g : rp.groups) {
        int64_t item0 = 0, blk0 = 0;
        for (int32_t e = g.first; e < g.first + g.count; ++e) {
            tab_csr[e] = inst_entry(rp.csr_order[e], item0, blk0);
            item0 += probs[rp.csr_order[e]].n;
            blk0 += (probs[rp.csr_order[e]].n + 63) / 64;
        }
    }
    RelInst *d_all = at<RelInst>(ws, rp.o_tab_all), *d_csr = at<RelInst>(ws, rp.o_tab_csr);
    QPA_HIP(hipMemcpyAsync(d_all, tab_all.data(), sizeof(RelInst) * tab_all.size(),
                           hipMemcpyHostToDevice, st));
    QPA_HIP(hipMemcpyAsync(d_csr, tab_csr.data(), sizeof(RelInst) * tab_csr.size(),
                           hipMemcpyHostToDevice, st));
    // the host tables are read by the copies: wait for them before they go out of scope
    QPA_HIP(hipStreamSynchronize(st));

    const int64_t Rp = rp.Rp;
    const int32_t T = params->steps, R = params->replicas;
    const size_t V = rp.vec_bytes();
    const size_t VN = (size_t)rp.rows * (size_t)Rp;      // floats per vector
    float *X[2] = {at<float>(ws, rp.o_x0), at<float>(ws, rp.o_x1)};
    float *M = at<float>(ws, rp.o_m);
    float *ckpt = at<float>(ws, rp.o_ckpt), *seg = at<float>(ws, rp.o_seg);
    float *xbar = at<float>(ws, rp.o_xbar), *yb = at<float>(ws, rp.o_yb);
    float *MU[2] = {at<float>(ws, rp.o_mu0), at<float>(ws, rp.o_mu1)};
    double *part = at<double>(ws, rp.o_part), *ploss = at<double>(ws, rp.o_ploss);
    auto slot_x = [&](int32_t sidx) { return seg + (size_t)3 * VN * (size_t)sidx; };
    auto slot_m = [&](int32_t sidx) { return slot_x(sidx) + VN; };
    auto slot_f = [&](int32_t sidx) { return slot_x(sidx) + 2 * VN; };

    RelArgs base{};
    base.Rp = Rp;
    base.R = R;
    base.nblk = rp.nblk;
    base.lam = lam;
    base.eta = params->eta;
    base.alpha = params->alpha;
    base.scale = scale;
    // The state pointers of a dense instance's launch point at its first row.
    auto shifted = [&](const RelArgs &a, int64_t row0) {
        RelArgs b = a;
        const int64_t o = row0 * Rp;
        auto sh = [&](auto *p) { return p ? p + o : p; };
        b.xi = sh(a.xi);
        b.mi = sh(a.mi);
        b.xo = sh(a.xo);
        b.mo = sh(a.mo);
        b.fo = sh(a.fo);
        b.sx = sh(a.sx);
        b.sm = sh(a.sm);
        b.sf = sh(a.sf);
        b.mu_in = sh(a.mu_in);
        b.mu_out = sh(a.mu_out);
        b.yb = sh(a.yb);
        b.xbar = sh(a.xbar);
        return b;
    };
    // One launch mode over every instance: the gather launches of the CSR groups and the
    // tiled products of the dense instances, each on its own partial slots.
    auto over_all = [&](int32_t mode, const RelArgs &a) -> qpa_status {
        for (const auto &g : rp.groups) {
            RelArgs b = a;
            b.slot0 = g.slot0;
            QPA_HIP(launch_rel_gather(mode, d_csr + g.first, g.count, g.blocks, rp.C, g.wdt,
                                      g.idt, b, st));
        }
        for (int32_t q = 0; q < count; ++q) {
            if (rp.dense_slot[q] < 0) continue;
            RelArgs b = shifted(a, rp.row0[q]);
            b.slot0 = rp.dense_slot[q];
            const char *wsq = at<char>(ws, rp.base[q]);
            QPA_HIP(launch_rel_tiles(mode, probs[q].n, at<float>(const_cast<char *>(wsq),
                                                                 rp.inst[q].o_Jf),
                                     at<float>(const_cast<char *>(wsq), rp.inst[q].o_bf), b,
                                     st));
        }
        return QPA_OK;
    };
    auto fwd = [&](int32_t t, const float *xi, const float *mi, float *xo, float *mo,
                   float *fo) {
        RelArgs a = base;
        a.t_f = t;
        a.xi = xi;
        a.mi = mi;
        a.xo = xo;
        a.mo = mo;
        a.fo = fo;
        return over_all(REL_MODE_FWD, a);
    };

    // initial state of every instance (seed + instance index), padding replicas zero
    for (int32_t q = 0; q < count; ++q) {
        const int64_t o = rp.row0[q] * Rp;
        QPA_HIP(launch_init_state(probs[q].n, R, params->seed + (uint64_t)q, params->sigma0,
                                  X[0] + o, M + o, 1, Rp, Rp, probs[q].n, st));
    }
    if (grads) QPA_HIP(launch_rel_fill(part, (int64_t)3 * rp.nblk * std::max(T, 1), st));
    QPA_HIP(launch_rel_fill(ploss, rp.nblk, st));
    // forward pass, keeping (x, m) at the first step of every segment
    for (int32_t t = 0; t < T; ++t) {
        if (grads && t % k == 0) {
            float *c = ckpt + (size_t)2 * VN * (size_t)(t / k);
            QPA_HIP(hipMemcpyAsync(c, X[t & 1], V, hipMemcpyDeviceToDevice, st));
            QPA_HIP(hipMemcpyAsync(c + VN, M, V, hipMemcpyDeviceToDevice, st));
        }
        s = fwd(t, X[t & 1], M, X[(t + 1) & 1], M, nullptr);
        if (s != QPA_OK) return s;
    }
    {
        RelArgs a = base;
        a.xi = X[T & 1];
        a.xbar = xbar;
        a.part = ploss;
        s = over_all(REL_MODE_LOSS, a);
        if (s != QPA_OK) return s;
    }
    if (grads && T > 0) {
        QPA_HIP(hipMemsetAsync(MU[0], 0, V, st));    // mu_{T+1} = 0
        int cur = 0;
        for (int32_t c = rp.nseg - 1; c >= 0; --c) {
            const int32_t t0 = c * k, t1 = std::min(T, t0 + k);
            const float *cp = ckpt + (size_t)2 * VN * (size_t)c;
            QPA_HIP(hipMemcpyAsync(slot_x(0), cp, V, hipMemcpyDeviceToDevice, st));
            QPA_HIP(hipMemcpyAsync(slot_m(0), cp + VN, V, hipMemcpyDeviceToDevice, st));
            for (int32_t t = t0; t < t1; ++t) {
                const int32_t q = t - t0;
                s = fwd(t, slot_x(q), slot_m(q), slot_x(q + 1), slot_m(q + 1), slot_f(q));
                if (s != QPA_OK) return s;
            }
            {   // A(t1 - 1) alone, element-wise over all rows
                RelArgs a = base;
                a.t_a = t1 - 1;
                a.sx = slot_x(t1 - 1 - t0);
                a.sm = slot_m(t1 - 1 - t0);
                a.sf = slot_f(t1 - 1 - t0);
                a.xbar = xbar;
                a.mu_in = MU[cur];
                a.mu_out = MU[cur ^ 1];
                a.yb = yb;
                a.part = part + (size_t)3 * rp.nblk * (size_t)(t1 - 1);
                a.slot0 = 0;
                QPA_HIP(launch_rel_gather(REL_MODE_A, d_all, count, rp.blocks_all, rp.C, 0, 0,
                                          a, st));
                cur ^= 1;
            }
            for (int32_t t = t1 - 1; t > t0; --t) {    // B(t), then A(t - 1)
                RelArgs a = base;
                a.t_f = t;
                a.t_a = t - 1;
                a.sx = slot_x(t - 1 - t0);
                a.sm = slot_m(t - 1 - t0);
                a.sf = slot_f(t - 1 - t0);
                a.mu_in = MU[cur];
                a.mu_out = MU[cur ^ 1];
                a.yb = yb;
                a.part = part + (size_t)3 * rp.nblk * (size_t)(t - 1);
                s = over_all(REL_MODE_BA, a);
                if (s != QPA_OK) return s;
                cur ^= 1;
            }
            {   // B(t0): xbar_{t0} for the segment before
                RelArgs a = base;
                a.t_f = t0;
                a.mu_in = MU[cur];
                a.yb = yb;
                a.xbar = xbar;
                s = over_all(REL_MODE_B, a);
                if (s != QPA_OK) return s;
            }
        }
    }
    QPA_HIP(launch_rel_finish(T, rp.nblk, part, ploss, loss, grads ? d_eta : nullptr,
                              grads ? d_alpha : nullptr, grads ? d_lambda : nullptr, st));
    return QPA_OK;
}

}  // namespace
}  // namespace qpa

extern "C" {

qpa_status qpa_workspace_size_relaxed_batch(qpa_ctx *ctx, int32_t count,
                                            const qpa_problem *problems,
                                            const qpa_params *params, int32_t ckpt_every,
                                            size_t *bytes) {
    if (!bytes) return fail(ctx, QPA_E_ARG, "bytes is NULL");
    qpa_status s = check_params(ctx, params);
    if (s != QPA_OK) return s;
    RelPlan rp;
    s = make_rel_plan(ctx, count, problems, *params, ckpt_every, rp);
    if (s != QPA_OK) return s;
    *bytes = rp.total;
    return QPA_OK;
}

qpa_status qpa_workspace_size_relaxed(qpa_ctx *ctx, const qpa_problem *problem,
                                      const qpa_params *params, int32_t ckpt_every,
                                      size_t *bytes) {
    return qpa_workspace_size_relaxed_batch(ctx, 1, problem, params, ckpt_every, bytes);
}

qpa_status qpa_relaxed_grad_batch(qpa_ctx *ctx, int32_t count, const qpa_problem *problems,
                                  const qpa_params *params, int32_t ckpt_every, double scale,
                                  void *workspace, size_t workspace_bytes, void *stream,
                                  double *loss, double *d_eta, double *d_alpha,
                                  double *d_lambda) {
    return relaxed_run(ctx, count, problems, params, ckpt_every, scale, workspace,
                       workspace_bytes, static_cast<hipStream_t>(stream), loss, d_eta, d_alpha,
                       d_lambda);
}

qpa_status qpa_relaxed_grad(qpa_ctx *ctx, const qpa_problem *problem, const qpa_params *params,
                            int32_t ckpt_every, double scale, void *workspace,
                            size_t workspace_bytes, void *stream, double *loss, double *d_eta,
                            double *d_alpha, double *d_lambda) {
    return relaxed_run(ctx, 1, problem, params, ckpt_every, scale, workspace, workspace_bytes,
                       static_cast<hipStream_t>(stream), loss, d_eta, d_alpha, d_lambda);
}

qpa_status qpa_workspace_size_batch(qpa_ctx *ctx, int32_t count, const qpa_problem *problems,
                                    const qpa_params *params, size_t *bytes) {
    if (!bytes) return fail(ctx, QPA_E_ARG, "bytes is NULL");
    qpa_status s = check_batch_params(ctx, params);
    if (s != QPA_OK) return s;
    BatchPlan bp;
    s = make_batch_plan(ctx, count, problems, *params, bp);
    if (s != QPA_OK) return s;
    *bytes = bp.total;
    return QPA_OK;
}

namespace {
constexpr int AUX_STREAMS = 4;

// Work enqueued on ctx->aux after this starts after everything already on `st`.
qpa_status aux_fork(qpa_ctx *ctx, hipStream_t st) {
    if (ctx->aux.empty()) {
        for (int i = 0; i < AUX_STREAMS; ++i) {
            hipStream_t a = nullptr;
            QPA_HIP(hipStreamCreateWithFlags(&a, hipStreamNonBlocking));
            ctx->aux.push_back(a);
        }
        for (int i = 0; i <= AUX_STREAMS; ++i) {
            hipEvent_t ev = nullptr;
            QPA_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            ctx->aux_ev.push_back(ev);
        }
    }
    QPA_HIP(hipEventRecord(ctx->aux_ev[0], st));
    for (auto a : ctx->aux) QPA_HIP(hipStreamWaitEvent(a, ctx->aux_ev[0], 0));
    return QPA_OK;
}

// Work enqueued on `st` after this starts after everything enqueued on ctx->aux.
qpa_status aux_join(qpa_ctx *ctx, hipStream_t st) {
    for (size_t i = 0; i < ctx->aux.size(); ++i) {
        QPA_HIP(hipEventRecord(ctx->aux_ev[1 + i], ctx->aux[i]));
        QPA_HIP(hipStreamWaitEvent(st, ctx->aux_ev[1 + i], 0));
    }
    return QPA_OK;
}

// Joins the auxiliary streams into `st` when a forked section is left early (an error
// return), so that nothing the caller orders after the call can overtake their work.
struct AuxGuard {
    qpa_ctx *ctx;
    hipStream_t st;
    bool open = true;
    ~AuxGuard() {
        if (!open) return;
        const std::string keep = ctx->err;     // the join must not replace the message
        (void)aux_join(ctx, st);
        ctx->err = keep;
    }
    qpa_status close() {
        open = false;
        return aux_join(ctx, st);
    }
};

// Issues body(k, stream) for instances 0 .. count-1 between aux_fork and aux_join:
// instance k goes to auxiliary stream k mod (number of streams), and each stream's
// instances are issued in order from a host thread of its own (the calling thread takes
// the first stream), since the host-side cost of the many small launches, not the GPU,
// bounds these sections.  body returns the first HIP error of its instance; a failing
// thread stops issuing, and the error of the lowest failing instance is reported.  body
// touches no shared state of the context.
extern "C++" {
template <class F>
qpa_status aux_issue(qpa_ctx *ctx, int32_t count, const char *what, F &&body) {
    const int32_t A = std::max<int32_t>(1, std::min<int32_t>((int32_t)ctx->aux.size(), count));
    std::vector<int32_t> bad_k(A, INT32_MAX);
    std::vector<hipError_t> bad_e(A, hipSuccess);
    auto share = [&](int32_t a) {
        hipError_t e = a == 0 ? hipSuccess : hipSetDevice(ctx->device);
        for (int32_t k = a; k < count && e == hipSuccess; k += A) {
            e = body(k, ctx->aux[a]);
            if (e != hipSuccess) bad_k[a] = k;
        }
        if (e != hipSuccess && bad_k[a] == INT32_MAX) bad_k[a] = a;
        bad_e[a] = e;
    };
    std::vector<std::thread> th;
    int32_t started = 1;
    try {
        for (; started < A; ++started) th.emplace_back(share, started);
    } catch (...) {
        // no thread for the remaining shares: the calling thread issues them
    }
    share(0);
    for (int32_t a = started; a < A; ++a) share(a);
    for (auto &t : th) t.join();
    int32_t worst = -1;
    for (int32_t a = 0; a < A; ++a)
        if (bad_e[a] != hipSuccess && (worst < 0 || bad_k[a] < bad_k[worst])) worst = a;
    if (worst < 0) return QPA_OK;
    return fail(ctx, QPA_E_DEVICE, "instance %d: %s: %s", bad_k[worst], what,
                hipGetErrorString(bad_e[worst]));
}
}  // extern "C++"
}  // namespace

qpa_status qpa_solve_batch(qpa_ctx *ctx, int32_t count, const qpa_problem *problems,
                           const qpa_params *params, void *workspace, size_t workspace_bytes,
                           void *stream, const qpa_outputs *out) {
    if (!ctx) return QPA_E_ARG;
    ctx->err.clear();
    ctx->batch_paths.clear();
    qpa_status s = check_batch_params(ctx, params);
    if (s != QPA_OK) return s;
    BatchPlan bp;
    s = make_batch_plan(ctx, count, problems, *params, bp);
    if (s != QPA_OK) return s;
    if (!workspace) return fail(ctx, QPA_E_ARG, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(workspace) % ALIGN) != 0)
        return fail(ctx, QPA_E_ARG, "workspace must be %zu-byte aligned", ALIGN);
    if (workspace_bytes < bp.total)
        return fail(ctx, QPA_E_WORKSPACE, "workspace has %zu bytes, %zu needed", workspace_bytes,
                    bp.total);
    if (!out) return fail(ctx, QPA_E_ARG, "out is NULL");
    for (int32_t k = 0; k < count; ++k)
        if (!out[k].energy || !out[k].best)
            return fail(ctx, QPA_E_ARG, "instance %d: outputs.energy and outputs.best are required",
                        k);
    QPA_HIP(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(workspace);
    s = upload_schedule(ctx, *params, reinterpret_cast<float *>(ws + bp.o_lam), st);
    if (s != QPA_OK) return s;

    // canonicalise + validate every instance (instances spread over the context's
    // auxiliary streams: their launches are small and independent), each also writing its
    // scalars into one array, then one read-back of that array
    std::vector<CanonScalars> hsc(count);
    CanonScalars *scall = reinterpret_cast<CanonScalars *>(ws + bp.o_scall);
    // integer instances on the wave-per-row pass with a one-launch finalisation are
    // canonicalised by batched launches from a table (once per coupling/index type pair)
    struct CanonGroup {
        qpa_dtype w, i;
        int32_t first, count;
        int64_t max_n;
    };
    std::vector<CanonTask> ctasks;
    std::vector<CanonGroup> cgroups;
    std::vector<char> canon_b(count, 0);
    for (qpa_dtype wt : {QPA_I8, QPA_I16, QPA_I32})
        for (qpa_dtype xt : {QPA_I16, QPA_I32}) {
            CanonGroup g{wt, xt, (int32_t)ctasks.size(), 0, 0};
            for (int32_t k = 0; k < count; ++k) {
                const qpa_problem &p = problems[k];
                if (p.coupling_dtype != wt || p.index_dtype != xt || !csr_rows_by_wave(p) ||
                    p.n > CANON_ROWS_PER_PART)
                    continue;
                const Plan &pl = bp.inst[k];
                char *iw = ws + bp.base[k];
                CanonTask t{};
                t.rp = p.row_ptr;
                t.col = p.col;
                t.w = p.weights;
                t.lin = p.linear;
                t.lin_dt = p.linear_dtype;
                t.is_qubo = p.kind == QPA_KIND_QUBO ? 1 : 0;
                t.is_int = dtype_is_int(p.coupling_dtype) &&
                           (p.linear == nullptr || dtype_is_int(p.linear_dtype));
                t.n = p.n;
                t.nnz = p.nnz;
                t.b_f32 = at<float>(iw, pl.o_bf);
                t.b_i64 = at<int64_t>(iw, pl.o_bi);
                t.b_f64 = at<double>(iw, pl.o_bd);
                t.row_abs = at<double>(iw, pl.o_rabs);
                t.row_max = at<double>(iw, pl.o_rmax);
                t.row_k = at<double>(iw, pl.o_rk);
                t.sc = at<CanonScalars>(iw, pl.o_sc);
                t.mirror = scall + k;
                ctasks.push_back(t);
                canon_b[k] = 1;
                ++g.count;
                g.max_n = std::max(g.max_n, p.n);
            }
            if (g.count) cgroups.push_back(g);
        }
    // one pinned block: the scalars' read-back, then the table
    const size_t cbytes = sizeof(CanonTask) * ctasks.size();
    char *stage = nullptr;
    s = host_stage(ctx, sizeof(CanonScalars) * (size_t)count + cbytes, &stage);
    if (s != QPA_OK) return s;
    CanonScalars *pinned = reinterpret_cast<CanonScalars *>(stage);
    CanonTask *ptab = reinterpret_cast<CanonTask *>(pinned + count);
    std::copy(ctasks.begin(), ctasks.end(), ptab);
    s = aux_fork(ctx, st);
    if (s != QPA_OK) return s;
    AuxGuard g0{ctx, st};
    if (!ctasks.empty()) {
        const CanonTask *dt = reinterpret_cast<const CanonTask *>(ws + bp.o_canon);
        hipError_t e = hipMemcpyAsync(ws + bp.o_canon, ptab, cbytes, hipMemcpyHostToDevice, st);
        for (const CanonGroup &g : cgroups)
            if (e == hipSuccess)
                e = launch_canon_batch(dt + g.first, g.count, g.w, g.i, g.max_n, st);
        if (e != hipSuccess)
            s = fail(ctx, QPA_E_DEVICE, "canonicalisation: %s", hipGetErrorString(e));
    }
    if (s == QPA_OK) s = aux_issue(ctx, count, "canonicalisation", [&](int32_t k, hipStream_t ak) {
        if (canon_b[k]) return hipSuccess;
        const Plan &pl = bp.inst[k];
        void *iw = ws + bp.base[k];
        return launch_canon_csr(problems[k], at<float>(iw, pl.o_bf), at<int64_t>(iw, pl.o_bi),
                                at<double>(iw, pl.o_bd), at<double>(iw, pl.o_rabs),
                                at<double>(iw, pl.o_rmax), at<double>(iw, pl.o_rk),
                                at<double>(iw, pl.o_cpart), at<CanonScalars>(iw, pl.o_sc), ak,
                                scall + k);
    });
    const qpa_status sj = g0.close();
    if (s == QPA_OK) s = sj;
    hipError_t se = hipSuccess;
    if (s == QPA_OK)
        se = hipMemcpyAsync(pinned, scall, sizeof(CanonScalars) * (size_t)count,
                            hipMemcpyDeviceToHost, st);
    const hipError_t se2 = hipStreamSynchronize(st);
    if (se == hipSuccess) se = se2;
    if (s != QPA_OK) return s;
    for (int32_t k = 0; k < count; ++k) hsc[k] = pinned[k];
    if (se != hipSuccess)
        return fail(ctx, QPA_E_DEVICE, "synchronise failed: %s", hipGetErrorString(se));
    for (int32_t k = 0; k < count; ++k) {
        const int32_t f = hsc[k].flags;
        if (f & (FLAG_SHAPE | FLAG_UNSORTED))
            return fail(ctx, QPA_E_SHAPE, "instance %d: CSR structure invalid", k);
        if (f & FLAG_ASYM) return fail(ctx, QPA_E_ASYM, "instance %d: couplings not symmetric", k);
        if (f & FLAG_RANGE)
            return fail(ctx, QPA_E_RANGE, "instance %d: integer row bound %.0f >= 2^24", k,
                        hsc[k].max_row);
    }

    // dense tiles for the candidates whose couplings are exact in BF16: int8 tiles for
    // integer weights with |w| <= 127 (exact int32 sums), BF16 tiles otherwise
    const int64_t R = params->replicas;
    std::vector<char> is_dense(count, 0);
    std::vector<MfmaTile> tiles, tiles8;
    std::vector<std::vector<MfmaTile>> itiles(count);
    // int8 slots (np <= 65536) are set up by batched launches below, the others per
    // instance on the auxiliary streams
    std::vector<char> slot8(count, 0);
    for (int32_t k = 0; k < count; ++k) {
        const DenseSlot &ds = bp.dense[k];
        if (ds.cand && bp.inst[k].is_int && hsc[k].max_abs <= 127.0 &&
            problems[k].coupling_dtype != QPA_F32 && ds.np <= 65536)
            slot8[k] = 1;
    }
    s = aux_fork(ctx, st);
    if (s != QPA_OK) return s;
    AuxGuard g1{ctx, st};
    s = aux_issue(ctx, count, "tile set-up", [&](int32_t k, hipStream_t ak) -> hipError_t {
        const DenseSlot &ds = bp.dense[k];
        if (!ds.cand) return hipSuccess;
        if (bp.inst[k].is_int && hsc[k].max_abs > 256.0) return hipSuccess;
        const bool i8 = bp.inst[k].is_int && hsc[k].max_abs <= 127.0 &&
                        problems[k].coupling_dtype != QPA_F32;
        is_dense[k] = i8 ? 2 : 1;
        const Plan &pl = bp.inst[k];
        char *iw = ws + bp.base[k];
        const qpa_problem &p = problems[k];
        uint16_t *Jb = reinterpret_cast<uint16_t *>(ws + ds.o_Jb);
        float *bfp = reinterpret_cast<float *>(ws + ds.o_bfp);
        float *dx = reinterpret_cast<float *>(ws + ds.o_x);
        float *dm = reinterpret_cast<float *>(ws + ds.o_m);
        uint32_t *s0 = reinterpret_cast<uint32_t *>(ws + ds.o_s0);
        uint32_t *s1 = reinterpret_cast<uint32_t *>(ws + ds.o_s1);
        const CanonScalars *sc = at<CanonScalars>(iw, pl.o_sc);
        if (!slot8[k]) {        // int8 slots: matrix, field and state by the batched launches
            hipError_t e = i8 ? launch_csr_to_i8(p, ds.np, reinterpret_cast<int8_t *>(Jb), ak)
                              : launch_csr_to_bf16(p, ds.np, sc, Jb, ak);
            if (e == hipSuccess)
                e = launch_pad_f32(p.n, ds.np, at<float>(iw, pl.o_bf), bfp, ak);
            if (e == hipSuccess)
                e = launch_init_state(p.n, R, params->seed + (uint64_t)k, params->sigma0, dx,
                                      dm, ds.np, 1, ds.Rp, ds.np, ak);
            if (e == hipSuccess)
                e = i8 ? launch_mfma_pack_spins_i8(ds.Rp, ds.np, dx,
                                                   reinterpret_cast<uint8_t *>(s0), ak)
                       : launch_mfma_pack_spins(ds.Rp, ds.np, dx, s0, ak);
            if (e != hipSuccess) return e;
        }
        std::vector<MfmaTile> &tv = itiles[k];
        // BF16: tiles of 128 replicas x 128 variables over the padded replicas; int8: 64 x
        // 256 over the replicas up to R (a tile past them would hold padding only)
        const int64_t bm = i8 ? MF_BM8 : MF_BM, bn = i8 ? MF_BN8 : MF_BN;
        const int64_t nrb = i8 ? (R + MF_BM8 - 1) / MF_BM8 : ds.Rp / MF_BM;
        tv.reserve((size_t)nrb * (size_t)(ds.np / bn));
        for (int64_t rb = 0; rb < nrb; ++rb)
            for (int64_t ib = 0; ib < ds.np / bn; ++ib) {
                MfmaTile tl{};
                tl.Jb = Jb;
                tl.b = bfp;
                tl.sc = sc;
                tl.s0 = s0;
                tl.s1 = s1;
                tl.x = dx;
                tl.m = dm;
                tl.np = ds.np;
                tl.Rp = ds.Rp;
                tl.I0 = ib * bn;
                tl.R0 = rb * bm;
                tl.rlive = R;
                tv.push_back(tl);
            }
        return hipSuccess;
    });
    const qpa_status sj1 = g1.close();
    if (s == QPA_OK) s = sj1;
    if (s != QPA_OK) return s;

    // batched set-up of the int8 slots: a table uploaded once, the matrix once per
    // coupling/index type pair, then x0, m0, byte spins and padded field in one launch
    {
        std::vector<SlotInitTask> it8;
        struct SlotGroup {
            qpa_dtype w, i;
            int32_t first, count;
            int64_t max_np;
        };
        std::vector<SlotGroup> groups;
        int64_t max_elems = 0;
        for (qpa_dtype wt : {QPA_I8, QPA_I16, QPA_I32})
            for (qpa_dtype xt : {QPA_I16, QPA_I32}) {
                SlotGroup g{wt, xt, (int32_t)it8.size(), 0, 0};
                for (int32_t k = 0; k < count; ++k) {
                    const qpa_problem &p = problems[k];
                    if (!slot8[k] || p.coupling_dtype != wt || p.index_dtype != xt) continue;
                    const DenseSlot &ds = bp.dense[k];
                    const Plan &pl = bp.inst[k];
                    char *iw = ws + bp.base[k];
                    SlotInitTask t{};
                    t.rp = p.row_ptr;
                    t.col = p.col;
                    t.w = p.weights;
                    t.bf = at<float>(iw, pl.o_bf);
                    t.J8 = reinterpret_cast<int8_t *>(ws + ds.o_Jb);
                    t.bfp = reinterpret_cast<float *>(ws + ds.o_bfp);
                    t.x = reinterpret_cast<float *>(ws + ds.o_x);
                    t.m = reinterpret_cast<float *>(ws + ds.o_m);
                    t.s8 = reinterpret_cast<uint8_t *>(ws + ds.o_s0);
                    t.n = p.n;
                    t.np = ds.np;
                    t.R = R;
                    t.Rp = ds.Rp;
                    t.seed = params->seed + (uint64_t)k;
                    it8.push_back(t);
                    ++g.count;
                    g.max_np = std::max(g.max_np, ds.np);
                    max_elems = std::max(max_elems, ds.Rp * ds.np);
                }
                if (g.count) groups.push_back(g);
            }
        if (!it8.empty()) {
            const size_t bytes = sizeof(SlotInitTask) * it8.size();
            SlotInitTask *h = nullptr;
            QPA_HIP(hipHostMalloc((void **)&h, bytes));
            std::copy(it8.begin(), it8.end(), h);
            hipError_t e = hipMemcpyAsync(ws + bp.o_slot, h, bytes, hipMemcpyHostToDevice, st);
            const hipError_t e2 = hipStreamSynchronize(st);
            (void)hipHostFree(h);
            if (e == hipSuccess) e = e2;
            if (e != hipSuccess)
                return fail(ctx, QPA_E_DEVICE, "slot table upload: %s", hipGetErrorString(e));
            const SlotInitTask *dt = reinterpret_cast<const SlotInitTask *>(ws + bp.o_slot);
            for (const SlotGroup &g : groups)
                QPA_HIP(launch_csr_to_i8_batch(dt + g.first, g.count, g.w, g.i, g.max_np, st));
            QPA_HIP(launch_slot_init_batch(dt, (int32_t)it8.size(), max_elems, params->sigma0,
                                           st));
        }
    }

    // int8 slots whose 16 x 128 blocks hold at most I8S_BLOCK_MAX nonzeros run as sparse
    // int8 tiles: their entry lists go into the second half of the slot's coupling buffer
    // (J8 takes np^2 of its 2 np^2 bytes; offsets, then entries)
    {
        std::vector<I8sTask> ts;
        std::vector<int32_t> who;
        int64_t max_np = 0;
        for (int32_t k = 0; k < count; ++k) {
            if (is_dense[k] != 2) continue;
            const DenseSlot &ds = bp.dense[k];
            char *jb = ws + ds.o_Jb;
            const size_t np2 = (size_t)(ds.np * ds.np);
            const size_t o_cnt = align_up(np2);
            const size_t o_e = o_cnt + align_up(sizeof(int32_t) * (size_t)(i8s_blocks(ds.np) + 1));
            I8sTask t{};
            t.J8 = reinterpret_cast<const int8_t *>(jb);
            t.cnt = reinterpret_cast<int32_t *>(jb + o_cnt);
            t.E = reinterpret_cast<uint32_t *>(jb + o_e);
            t.stats = reinterpret_cast<int32_t *>(ws + bp.o_i8s_stats) + 2 * ts.size();
            t.np = ds.np;
            ts.push_back(t);
            who.push_back(k);
            max_np = std::max(max_np, ds.np);
        }
        if (!ts.empty()) {
            const size_t tb = sizeof(I8sTask) * ts.size(), sb = 2 * sizeof(int32_t) * ts.size();
            char *h = nullptr;
            QPA_HIP(hipHostMalloc((void **)&h, tb + sb));
            std::copy(ts.begin(), ts.end(), reinterpret_cast<I8sTask *>(h));
            const I8sTask *dt = reinterpret_cast<const I8sTask *>(ws + bp.o_i8s_tab);
            const int32_t nt = (int32_t)ts.size();
            hipError_t e = hipMemcpyAsync(ws + bp.o_i8s_tab, h, tb, hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = launch_i8s_count(dt, nt, max_np, st);
            if (e == hipSuccess) e = launch_i8s_scan(dt, nt, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(h + tb, ws + bp.o_i8s_stats, sb, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = launch_i8s_fill(dt, nt, max_np, st);
            const hipError_t e2 = hipStreamSynchronize(st);
            if (e == hipSuccess) e = e2;
            std::vector<int32_t> stats(2 * ts.size());
            std::copy(reinterpret_cast<int32_t *>(h + tb),
                      reinterpret_cast<int32_t *>(h + tb) + 2 * ts.size(), stats.begin());
            (void)hipHostFree(h);
            if (e != hipSuccess)
                return fail(ctx, QPA_E_DEVICE, "sparse int8 tiles: %s", hipGetErrorString(e));
            for (size_t j = 0; j < ts.size(); ++j) {
                if (stats[2 * j] > I8S_BLOCK_MAX) continue;
                const int32_t k = who[j];
                const DenseSlot &ds = bp.dense[k];
                const size_t room = 2 * (size_t)(ds.np * ds.np) -
                                    (size_t)(reinterpret_cast<char *>(ts[j].E) - (ws + ds.o_Jb));
                if ((size_t)stats[2 * j + 1] * sizeof(uint32_t) > room)
                    return fail(ctx, QPA_E_DEVICE, "instance %d: sparse int8 entries overflow", k);
                is_dense[k] = 3;
                for (MfmaTile &tl : itiles[k]) {
                    tl.E = ts[j].E;
                    tl.O = ts[j].cnt;
                }
            }
        }
    }
    std::vector<MfmaTile> tiles8s;
    for (int32_t k = 0; k < count; ++k) {
        std::vector<MfmaTile> &dst = is_dense[k] == 3 ? tiles8s : is_dense[k] == 2 ? tiles8 : tiles;
        dst.insert(dst.end(), itiles[k].begin(), itiles[k].end());
    }

    // densified integer instances (n <= EBITS_MAX_N) are scored by batched launches (one
    // per kind; the energy kernels once per coupling/index type pair)
    struct ScoreGroup {
        qpa_dtype w, i;
        int32_t first, count;
        int64_t max_n, max_words;
    };
    std::vector<ScoreTask> stasks;
    std::vector<ScoreGroup> sgroups;
    std::vector<char> batched(count, 0);
    int64_t score_elems = 0, score_R = 0;
    for (qpa_dtype wt : {QPA_I8, QPA_I16, QPA_I32})
        for (qpa_dtype it : {QPA_I16, QPA_I32}) {
            ScoreGroup g{wt, it, (int32_t)stasks.size(), 0, 0, 0};
            for (int32_t k = 0; k < count; ++k) {
                const qpa_problem &p = problems[k];
                const Plan &pl = bp.inst[k];
                const bool is_int = dtype_is_int(p.coupling_dtype) &&
                                    (p.linear == nullptr || dtype_is_int(p.linear_dtype));
                if (!is_dense[k] || p.coupling_dtype != wt || p.index_dtype != it || !is_int ||
                    p.n > EBITS_MAX_N || energy_bits_blocks(p.n) > pl.eblk)
                    continue;
                const DenseSlot &ds = bp.dense[k];
                char *iw = ws + bp.base[k];
                const qpa_outputs &o = out[k];
                ScoreTask t{};
                t.x = reinterpret_cast<const float *>(ws + ds.o_x);
                t.ld_r = ds.np;
                t.n = p.n;
                t.R = pl.R;
                t.nblk = energy_bits_blocks(p.n);
                t.rp = p.row_ptr;
                t.col = p.col;
                t.w = p.weights;
                t.b_i64 = at<int64_t>(iw, pl.o_bi);
                t.sc = at<CanonScalars>(iw, pl.o_sc);
                t.spins = o.spins ? o.spins : at<int8_t>(iw, pl.o_sp);
                t.partial = at<double>(iw, pl.o_part);
                t.e_i64 = o.energy_i64 ? o.energy_i64 : at<int64_t>(iw, pl.o_ei);
                t.e_f64 = o.energy;
                t.best = o.best;
                t.words = reinterpret_cast<uint64_t *>(ws + ds.o_s1);   // free after the steps
                t.is_qubo = p.kind == QPA_KIND_QUBO ? 1 : 0;
                stasks.push_back(t);
                batched[k] = 1;
                ++g.count;
                g.max_n = std::max(g.max_n, t.n);
                g.max_words = std::max(g.max_words, t.R * ((t.n + 63) / 64));
                score_elems = std::max(score_elems, t.R * t.n);
                score_R = std::max(score_R, t.R);
            }
            if (g.count) sgroups.push_back(g);
        }
    // largest instances first so that the tail of each step is made of small tiles; the
    // int8 tiles follow the BF16 ones in the uploaded table
    auto by_size = [](const MfmaTile &a, const MfmaTile &b) { return a.np > b.np; };
    std::stable_sort(tiles.begin(), tiles.end(), by_size);
    std::stable_sort(tiles8.begin(), tiles8.end(), by_size);
    std::stable_sort(tiles8s.begin(), tiles8s.end(), by_size);
    tiles = by_compute_die(tiles);
    tiles8 = by_compute_die(tiles8);
    tiles8s = by_compute_die(tiles8s);
    const int32_t ntiles16 = (int32_t)tiles.size(), ntiles8 = (int32_t)tiles8.size(),
                  ntiles8s = (int32_t)tiles8s.size();
    tiles.insert(tiles.end(), tiles8.begin(), tiles8.end());
    tiles.insert(tiles.end(), tiles8s.begin(), tiles8s.end());

    // task table of the CSR instances, largest (most stored entries) first
    std::vector<std::pair<int64_t, BatchTask>> order;
    order.reserve(bp.ntasks);
    for (int32_t k = 0; k < count; ++k) {
        if (is_dense[k]) continue;
        const Plan &pl = bp.inst[k];
        char *iw = ws + bp.base[k];
        const qpa_problem &p = problems[k];
        for (int64_t g = 0; g < pl.Rp / 64; ++g) {
            BatchTask tk{};
            tk.n = p.n;
            tk.rp = p.row_ptr;
            tk.col = p.col;
            tk.w = p.weights;
            tk.col_dt = p.index_dtype;
            tk.w_dt = p.coupling_dtype;
            tk.is_int = pl.is_int ? 1 : 0;
            tk.skip_diag = pl.is_qubo ? 1 : 0;
            tk.b = at<float>(iw, pl.o_bf);
            tk.x = at<float>(iw, pl.o_x) + g * p.n * 64;
            tk.m = at<float>(iw, pl.o_m) + g * p.n * 64;
            tk.seed = params->seed + (uint64_t)k;
            tk.group = (int32_t)g;
            tk.nrep = (int32_t)std::min<int64_t>(64, R - 64 * g);
            order.push_back({p.nnz + p.n, tk});
        }
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<int64_t, BatchTask> &a,
                        const std::pair<int64_t, BatchTask> &b) { return a.first > b.first; });
    std::vector<BatchTask> tasks;
    tasks.reserve(order.size());
    for (auto &pr : order) tasks.push_back(pr.second);
    const size_t tbytes = sizeof(BatchTask) * tasks.size();
    const size_t lbytes = sizeof(MfmaTile) * tiles.size();
    const size_t sbytes = sizeof(ScoreTask) * stasks.size();
    char *hbuf = nullptr;
    s = host_stage(ctx, tbytes + lbytes + sbytes, &hbuf);
    if (s != QPA_OK) return s;
    std::copy(tasks.begin(), tasks.end(), reinterpret_cast<BatchTask *>(hbuf));
    std::copy(tiles.begin(), tiles.end(), reinterpret_cast<MfmaTile *>(hbuf + tbytes));
    std::copy(stasks.begin(), stasks.end(), reinterpret_cast<ScoreTask *>(hbuf + tbytes + lbytes));
    hipError_t ce = hipSuccess;
    if (tbytes) ce = hipMemcpyAsync(ws + bp.o_tasks, hbuf, tbytes, hipMemcpyHostToDevice, st);
    if (ce == hipSuccess && lbytes)
        ce = hipMemcpyAsync(ws + bp.o_tiles, hbuf + tbytes, lbytes, hipMemcpyHostToDevice, st);
    if (ce == hipSuccess && sbytes)
        ce = hipMemcpyAsync(ws + bp.o_score, hbuf + tbytes + lbytes, sbytes,
                            hipMemcpyHostToDevice, st);
    const hipError_t ce2 = hipStreamSynchronize(st);     // the staging block is idle again
    if (ce == hipSuccess) ce = ce2;
    if (ce != hipSuccess) return fail(ctx, QPA_E_DEVICE, "task upload: %s", hipGetErrorString(ce));

    const float *dlam = reinterpret_cast<const float *>(ws + bp.o_lam);
    // The sparse task kernel (a few workgroups for all steps, instances disjoint from the
    // tiles') runs beside the grouped tile launches: forked onto an auxiliary stream before
    // the step loop and joined back before the scoring.
    const bool beside = !tasks.empty() && !tiles.empty() && params->steps > 0;
    AuxGuard gt{ctx, st, beside};
    if (beside) {
        s = aux_fork(ctx, st);
        if (s != QPA_OK) return s;
    }
    if (!tasks.empty()) {
        hipStream_t ts = beside ? ctx->aux[0] : st;
        int cus = 0;
        QPA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
        const int32_t ntask = (int32_t)tasks.size();
        const int32_t blocks = (int32_t)std::min<int64_t>(ntask, (int64_t)cus * 4);
        qpa_ctx::Span sp{};
        if (ctx->prof) {
            QPA_HIP(take_event(ctx, &sp.a));
            QPA_HIP(take_event(ctx, &sp.b));
            QPA_HIP(hipEventRecord(sp.a, ts));
        }
        QPA_HIP(launch_csr_batch(reinterpret_cast<const BatchTask *>(ws + bp.o_tasks), ntask,
                                 reinterpret_cast<int32_t *>(ws + bp.o_counter), blocks,
                                 params->steps, dlam, params->eta, params->alpha, params->sigma0,
                                 bp.max_n, ts));
        if (ctx->prof) {
            QPA_HIP(hipEventRecord(sp.b, ts));
            sp.launches = 1;
            sp.path = QPA_PATH_BATCH_SPARSE;
            ctx->spans.push_back(sp);
        }
    }
    if (!tiles.empty() && params->steps > 0) {
        qpa_ctx::Span sp{};
        if (ctx->prof) {
            QPA_HIP(take_event(ctx, &sp.a));
            QPA_HIP(take_event(ctx, &sp.b));
            QPA_HIP(hipEventRecord(sp.a, st));
        }
        const MfmaTile *dt16 = reinterpret_cast<const MfmaTile *>(ws + bp.o_tiles);
        auto loop = [&](hipStream_t s_) -> qpa_status {
            for (int32_t t = 0; t < params->steps; ++t) {
                QPA_HIP(launch_mfma_grouped(dt16, ntiles16, t, dlam, params->eta, params->alpha,
                                            GK_BF16, s_));
                QPA_HIP(launch_mfma_grouped(dt16 + ntiles16, ntiles8, t, dlam, params->eta,
                                            params->alpha, GK_I8, s_));
                QPA_HIP(launch_mfma_grouped(dt16 + ntiles16 + ntiles8, ntiles8s, t, dlam,
                                            params->eta, params->alpha, GK_I8_SPARSE, s_));
            }
            return QPA_OK;
        };
        if (params->flags & QPA_SOLVE_GRAPH) {
            // the step loop's launches read only these host values (the tile table and
            // the schedule are device data written before the replay)
            std::vector<uint8_t> key;
            key_add(key, (int32_t)2);
            key_add(key, ws);
            key_add(key, bp.o_tiles);
            key_add(key, bp.o_lam);
            key_add(key, ntiles16);
            key_add(key, ntiles8);
            key_add(key, ntiles8s);
            key_add(key, params->steps);
            key_add(key, params->eta);
            key_add(key, params->alpha);
            s = run_graph(ctx, std::move(key), st, loop);
        } else {
            s = loop(st);
        }
        if (s != QPA_OK) return s;
        if (ctx->prof) {
            QPA_HIP(hipEventRecord(sp.b, st));
            sp.launches = (int64_t)params->steps * ((ntiles16 > 0) + (ntiles8 > 0) + (ntiles8s > 0));
            sp.path = QPA_PATH_BATCH_DENSE;
            ctx->spans.push_back(sp);
        }
    }
    if (beside) {
        s = gt.close();
        if (s != QPA_OK) return s;
    }

    // per instance: spins, optional state, exact energies, best replica (instances spread
    // over the auxiliary streams, joined back into the caller's stream at the end)
    s = aux_fork(ctx, st);
    if (s != QPA_OK) return s;
    AuxGuard g2{ctx, st};
    if (!stasks.empty()) {
        const ScoreTask *dst = reinterpret_cast<const ScoreTask *>(ws + bp.o_score);
        const int32_t ns = (int32_t)stasks.size();
        QPA_HIP(launch_export_spins_batch(dst, ns, score_elems, st));
        for (const ScoreGroup &g : sgroups)
            QPA_HIP(launch_energy_bits_batch(dst + g.first, g.count, g.w, g.i, g.max_n,
                                             g.max_words, st));
        QPA_HIP(launch_finalize_argmin_batch(dst, ns, score_R, st));
    }
    for (int32_t k = 0; k < count; ++k) {
        hipStream_t ak = ctx->aux[(size_t)k % ctx->aux.size()];
        const Plan &pl = bp.inst[k];
        char *iw = ws + bp.base[k];
        const qpa_problem &p = problems[k];
        const qpa_outputs &o = out[k];
        int8_t *spins = o.spins ? o.spins : at<int8_t>(iw, pl.o_sp);
        if (is_dense[k]) {
            const DenseSlot &ds = bp.dense[k];
            const float *dx = reinterpret_cast<const float *>(ws + ds.o_x);
            const float *dm = reinterpret_cast<const float *>(ws + ds.o_m);
            if (!batched[k]) QPA_HIP(launch_export_spins(p.n, R, dx, ds.np, 1, spins, ak));
            if (o.x) QPA_HIP(launch_copy_state(p.n, R, dx, ds.np, 1, o.x, p.n, 1, ak));
            if (o.m) QPA_HIP(launch_copy_state(p.n, R, dm, ds.np, 1, o.m, p.n, 1, ak));
        }
        for (int64_t g = 0; !is_dense[k] && g < pl.Rp / 64; ++g) {
            const int64_t rg = std::min<int64_t>(64, R - 64 * g);
            const float *xg = at<float>(iw, pl.o_x) + g * p.n * 64;
            const float *mg = at<float>(iw, pl.o_m) + g * p.n * 64;
            QPA_HIP(launch_export_spins(p.n, rg, xg, 1, 64, spins + g * 64 * p.n, ak));
            if (o.x) QPA_HIP(launch_copy_state(p.n, rg, xg, 1, 64, o.x + g * 64 * p.n, p.n, 1, ak));
            if (o.m) QPA_HIP(launch_copy_state(p.n, rg, mg, 1, 64, o.m + g * 64 * p.n, p.n, 1, ak));
        }
        if (batched[k]) continue;
        s = score(ctx, p, pl, iw, spins, o.energy, o.energy_i64, o.best, ak);
        if (s != QPA_OK) {
            std::string msg = "instance " + std::to_string(k) + ": " + ctx->err;
            return fail(ctx, s, "%s", msg.c_str());
        }
    }
    s = g2.close();
    if (s != QPA_OK) return s;
    ctx->batch_paths.assign(count, QPA_PATH_BATCH_SPARSE);
    for (int32_t k = 0; k < count; ++k)
        if (is_dense[k])
            ctx->batch_paths[k] = is_dense[k] == 3   ? QPA_PATH_BATCH_SPARSE_I8
                                  : is_dense[k] == 2 ? QPA_PATH_BATCH_DENSE_I8
                                                     : QPA_PATH_BATCH_DENSE;
    return QPA_OK;
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

// ---------------------------------------------------------------- SBM (App. B)
namespace {

qpa_status sbm_prologue(qpa_ctx *ctx, const qpa_problem *problem, const qpa_sbm_params *params,
                        void *ws, size_t ws_bytes, SbmPlan &sp) {
    if (!ctx) return QPA_E_ARG;
    ctx->err.clear();
    qpa_status s = check_problem(ctx, problem);
    if (s != QPA_OK) return s;
    s = check_sbm_params(ctx, params);
    if (s != QPA_OK) return s;
    sp = make_sbm_plan(*problem, *params, ctx->cus);
    if (!ws) return fail(ctx, QPA_E_ARG, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(ws) % ALIGN) != 0)
        return fail(ctx, QPA_E_ARG, "workspace must be %zu-byte aligned", ALIGN);
    if (ws_bytes < sp.total)
        return fail(ctx, QPA_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes,
                    sp.total);
    QPA_HIP(hipSetDevice(ctx->device));
    return QPA_OK;
}

// c0 into the workspace: the caller's value, or 1 / rho from the power method.
qpa_status sbm_set_c0(qpa_ctx *ctx, const qpa_problem &p, const qpa_sbm_params &s,
                      const SbmPlan &sp, void *ws, double *rho, hipStream_t st) {
    float *c0 = at<float>(ws, sp.o_c0);
    if (s.c0 > 0.0f && !rho) {
        QPA_HIP(launch_set_f32(c0, s.c0, st));
        return QPA_OK;
    }
    QPA_HIP(launch_power_method(p, s.power_iters, s.seed, at<double>(ws, sp.o_pv),
                                at<double>(ws, sp.o_pw), at<double>(ws, sp.o_pp),
                                at<double>(ws, sp.o_nrm), rho, s.c0 > 0.0f ? nullptr : c0, st));
    if (s.c0 > 0.0f) QPA_HIP(launch_set_f32(c0, s.c0, st));
    return QPA_OK;
}

// a(t) = a0 * ((float)t / (float)T) for every step, the expression the per-step launches
// evaluate, staged through the pinned schedule buffer.
qpa_status upload_sbm_schedule(qpa_ctx *ctx, const qpa_sbm_params &s, float *d_a,
                               hipStream_t st) {
    const int64_t T = s.steps;
    if (T == 0) return QPA_OK;
    if (ctx->host_lam_cap < (size_t)T) {
        if (ctx->host_lam) (void)hipHostFree(ctx->host_lam);
        ctx->host_lam = nullptr;
        QPA_HIP(hipHostMalloc((void **)&ctx->host_lam, sizeof(float) * (size_t)T));
        ctx->host_lam_cap = (size_t)T;
    }
    QPA_HIP(hipStreamSynchronize(st));
    for (int64_t t = 0; t < T; ++t) {
        volatile float frac = (float)t / (float)T;
        ctx->host_lam[t] = s.a0 * frac;
    }
    QPA_HIP(hipMemcpyAsync(d_a, ctx->host_lam, sizeof(float) * (size_t)T, hipMemcpyHostToDevice,
                           st));
    return QPA_OK;
}

// Steps t0 .. t1-1 from the positions in q0; returns the buffer holding the last ones.
qpa_status sbm_run(qpa_ctx *ctx, const qpa_problem &p, const qpa_sbm_params &s,
                   const SbmPlan &sp, void *ws, int32_t t0, int32_t t1, bool want_g,
                   hipStream_t st, float **q_last) {
    float *qa = at<float>(ws, sp.o_q0), *qb = at<float>(ws, sp.o_q1);
    *q_last = qa;
    if (t1 <= t0) return QPA_OK;
    const float *Jf = sp.base.o_Jf ? at<float>(ws, sp.base.o_Jf) : nullptr;
    const float *bf = at<float>(ws, sp.base.o_bf);
    const float *c0 = at<float>(ws, sp.o_c0);
    float *pm = at<float>(ws, sp.o_p), *g = at<float>(ws, sp.o_g);
    const bool resident = p.format == QPA_FMT_CSR && sp.Gres > 0;
    if (resident) {
        qpa_status us = upload_sbm_schedule(ctx, s, at<float>(ws, sp.o_atab), st);
        if (us != QPA_OK) return us;
    }
    qpa_ctx::Span sp_ev{};
    if (ctx->prof) {
        QPA_HIP(take_event(ctx, &sp_ev.a));
        QPA_HIP(take_event(ctx, &sp_ev.b));
        QPA_HIP(hipEventRecord(sp_ev.a, st));
    }
    if (resident) {
        QPA_HIP(launch_sbm_resident(p, sp.Gres, s.replicas, sp.Rp, bf, c0,
                                    at<float>(ws, sp.o_atab), s.a0, s.dt, qa, pm,
                                    want_g ? g : nullptr, t0, t1, st));
        if (ctx->prof) {
            QPA_HIP(hipEventRecord(sp_ev.b, st));
            sp_ev.launches = 1;
            sp_ev.path = QPA_PATH_SBM_CSR_RESIDENT;
            ctx->spans.push_back(sp_ev);
        }
        return QPA_OK;
    }
    auto loop = [&](hipStream_t s_) -> qpa_status {
        float *q_in = qa, *q_out = qb;
        for (int32_t t = t0; t < t1; ++t) {
            volatile float frac = (float)t / (float)s.steps;
            const float a = s.a0 * frac;
            QPA_HIP(launch_sbm_step(p, Jf, sp.Rp, bf, c0, a, s.a0, s.dt, q_in, q_out, pm,
                                    (want_g && t == t1 - 1) ? g : nullptr, s_));
            std::swap(q_in, q_out);
        }
        return QPA_OK;
    };
    qpa_status rs;
    if (s.flags & QPA_SOLVE_GRAPH) {
        std::vector<uint8_t> key;
        key_add(key, (int32_t)2);
        key_add(key, p);
        key_add(key, sp.Rp);
        key_add(key, sp.total);
        key_add(key, ws);
        key_add(key, s.a0);
        key_add(key, s.dt);
        key_add(key, s.steps);
        key_add(key, t0);
        key_add(key, t1);
        key_add(key, want_g);
        rs = run_graph(ctx, std::move(key), st, loop);
    } else {
        rs = loop(st);
    }
    if (rs != QPA_OK) return rs;
    if ((t1 - t0) & 1) std::swap(qa, qb);
    *q_last = qa;
    if (ctx->prof) {
        QPA_HIP(hipEventRecord(sp_ev.b, st));
        sp_ev.launches = t1 - t0;
        sp_ev.path = p.format == QPA_FMT_DENSE ? QPA_PATH_SBM_DENSE : QPA_PATH_SBM_CSR;
        ctx->spans.push_back(sp_ev);
    }
    return QPA_OK;
}

}  // namespace

qpa_status qpa_workspace_size_sbm(qpa_ctx *ctx, const qpa_problem *problem,
                                  const qpa_sbm_params *params, size_t *bytes) {
    if (!bytes) return fail(ctx, QPA_E_ARG, "bytes is NULL");
    qpa_status s = check_problem(ctx, problem);
    if (s != QPA_OK) return s;
    s = check_sbm_params(ctx, params);
    if (s != QPA_OK) return s;
    *bytes = make_sbm_plan(*problem, *params, 256).total;
    return QPA_OK;
}

qpa_status qpa_sbm_solve(qpa_ctx *ctx, const qpa_problem *problem, const qpa_sbm_params *params,
                         void *workspace, size_t workspace_bytes, void *stream,
                         const qpa_outputs *out) {
    SbmPlan sp;
    qpa_status s = sbm_prologue(ctx, problem, params, workspace, workspace_bytes, sp);
    if (s != QPA_OK) return s;
    if (!out || !out->energy || !out->best)
        return fail(ctx, QPA_E_ARG, "outputs.energy and outputs.best are required");
    hipStream_t st = static_cast<hipStream_t>(stream);
    void *ws = workspace;
    const Plan &pl = sp.base;
    s = canonicalise(ctx, *problem, pl, ws, st);
    if (s != QPA_OK) return s;
    const int64_t n = problem->n, R = params->replicas;
    float *q0 = at<float>(ws, sp.o_q0), *pm = at<float>(ws, sp.o_p);
    QPA_HIP(launch_init_state(n, R, params->seed, params->sigma0, q0, pm, 1, sp.Rp, sp.Rp, n,
                              st));
    s = sbm_set_c0(ctx, *problem, *params, sp, ws, nullptr, st);
    if (s != QPA_OK) return s;
    float *q = nullptr;
    s = sbm_run(ctx, *problem, *params, sp, ws, 0, params->steps, false, st, &q);
    if (s != QPA_OK) return s;
    int8_t *spins = out->spins ? out->spins : at<int8_t>(ws, pl.o_sp);
    QPA_HIP(launch_export_spins(n, R, q, 1, sp.Rp, spins, st));
    if (out->x) QPA_HIP(launch_copy_state(n, R, q, 1, sp.Rp, out->x, n, 1, st));
    if (out->m) QPA_HIP(launch_copy_state(n, R, pm, 1, sp.Rp, out->m, n, 1, st));
    return score(ctx, *problem, pl, ws, spins, out->energy, out->energy_i64, out->best, st);
}

qpa_status qpa_sbm_steps(qpa_ctx *ctx, const qpa_problem *problem, const qpa_sbm_params *params,
                         int32_t t0, int32_t t1, float *q_io, float *p_io, float *g_last,
                         void *workspace, size_t workspace_bytes, void *stream) {
    SbmPlan sp;
    qpa_status s = sbm_prologue(ctx, problem, params, workspace, workspace_bytes, sp);
    if (s != QPA_OK) return s;
    if (!q_io || !p_io) return fail(ctx, QPA_E_ARG, "q and p are required");
    if (t0 < 0 || t1 < t0 || t1 > params->steps)
        return fail(ctx, QPA_E_ARG, "need 0 <= t0 <= t1 <= steps (got %d, %d, %d)", t0, t1,
                    params->steps);
    hipStream_t st = static_cast<hipStream_t>(stream);
    void *ws = workspace;
    s = canonicalise(ctx, *problem, sp.base, ws, st);
    if (s != QPA_OK) return s;
    const int64_t n = problem->n, R = params->replicas;
    float *q0 = at<float>(ws, sp.o_q0), *pm = at<float>(ws, sp.o_p);
    if (sp.Rp != R) {
        // padding replicas start at zero; they never feed a live replica
        QPA_HIP(hipMemsetAsync(q0, 0, sizeof(float) * (size_t)(sp.Rp * n), st));
        QPA_HIP(hipMemsetAsync(pm, 0, sizeof(float) * (size_t)(sp.Rp * n), st));
    }
    QPA_HIP(launch_copy_state(n, R, q_io, n, 1, q0, 1, sp.Rp, st));
    QPA_HIP(launch_copy_state(n, R, p_io, n, 1, pm, 1, sp.Rp, st));
    s = sbm_set_c0(ctx, *problem, *params, sp, ws, nullptr, st);
    if (s != QPA_OK) return s;
    float *q = nullptr;
    s = sbm_run(ctx, *problem, *params, sp, ws, t0, t1, g_last != nullptr, st, &q);
    if (s != QPA_OK) return s;
    QPA_HIP(launch_copy_state(n, R, q, 1, sp.Rp, q_io, n, 1, st));
    QPA_HIP(launch_copy_state(n, R, pm, 1, sp.Rp, p_io, n, 1, st));
    if (g_last && t1 > t0)
        QPA_HIP(launch_copy_state(n, R, at<float>(ws, sp.o_g), 1, sp.Rp, g_last, n, 1, st));
    return QPA_OK;
}

qpa_status qpa_spectral_radius(qpa_ctx *ctx, const qpa_problem *problem,
                               const qpa_sbm_params *params, void *workspace,
                               size_t workspace_bytes, void *stream, double *rho) {
    SbmPlan sp;
    qpa_status s = sbm_prologue(ctx, problem, params, workspace, workspace_bytes, sp);
    if (s != QPA_OK) return s;
    if (!rho) return fail(ctx, QPA_E_ARG, "rho is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    s = canonicalise(ctx, *problem, sp.base, workspace, st);
    if (s != QPA_OK) return s;
    return sbm_set_c0(ctx, *problem, *params, sp, workspace, rho, st);
}

// ---------------------------------------------------------------- autotuning
namespace {
void record_choice(qpa_ctx *ctx, const qpa_problem &p, const qpa_params &a, int32_t choice) {
    const qpa_ctx::TuneKey k = tune_key(p, a);
    for (auto &e : ctx->tuned)
        if (e.first == k) {
            e.second = choice;
            return;
        }
    ctx->tuned.emplace_back(k, choice);
}
}  // namespace

qpa_status qpa_autotune(qpa_ctx *ctx, const qpa_problem *problem, const qpa_params *params,
                        int32_t probe_steps, void *workspace, size_t workspace_bytes,
                        void *stream, int32_t *choice, double *ms) {
    Plan pl;
    qpa_status s = prologue(ctx, problem, params, workspace, workspace_bytes, pl);
    if (s != QPA_OK) return s;
    if (problem->format != QPA_FMT_CSR)
        return fail(ctx, QPA_E_UNSUPPORTED, "autotuning covers sparse (CSR) problems");
    if (params->flags & (QPA_SOLVE_STREAMED | QPA_SOLVE_BINNED))
        return fail(ctx, QPA_E_ARG, "QPA_SOLVE_STREAMED or QPA_SOLVE_BINNED leaves nothing to choose");
    if (probe_steps < 1) return fail(ctx, QPA_E_ARG, "probe_steps must be >= 1");
    if (!choice) return fail(ctx, QPA_E_ARG, "choice is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    void *ws = workspace;
    s = upload_schedule(ctx, *params, at<float>(ws, pl.o_lam), st);
    if (s != QPA_OK) return s;
    s = canonicalise(ctx, *problem, pl, ws, st);
    if (s != QPA_OK) return s;
    const int32_t t1 = params->steps < probe_steps ? params->steps : probe_steps;
    float *x = at<float>(ws, pl.o_x), *m = at<float>(ws, pl.o_m);
    int64_t ld_r, ld_i;
    state_strides(pl, ld_r, ld_i);
    hipEvent_t e0, e1;
    QPA_HIP(hipEventCreate(&e0));
    QPA_HIP(hipEventCreate(&e1));
    const int cand[6] = {0, 1, 2, 4, 8, TUNE_BINNED};
    double best = -1.0;
    int32_t pick = 0;
    qpa_params a = *params;
    a.flags &= ~QPA_SOLVE_GRAPH;
    for (int c = 0; c < 6 && s == QPA_OK; ++c) {
        if (ms) ms[c] = -1.0;
        Plan q = pl;
        if (cand[c] == 0) {
            q.path = Path::Csr;
            q.G = q.Gs;
        } else if (cand[c] == TUNE_BINNED) {
            if (!pl.bin_ok) continue;
            q.path = Path::CsrBinned;
            q.G = q.Gs;
            s = bin_build(ctx, *problem, q, ws, st);
            if (s != QPA_OK) break;
        } else {
            if (!resident_ok(*problem, cand[c])) continue;
            q.path = Path::CsrResident;
            q.G = cand[c];
        }
        float took = 0.0f;
        for (int rep = 0; rep < 2 && s == QPA_OK; ++rep) {      // first run warms up
            hipError_t e = launch_init_state(q.n, q.R, params->seed, params->sigma0, x, m, ld_r,
                                             ld_i, q.Rp, q.np, st);
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            if (e != hipSuccess) {
                s = fail(ctx, QPA_E_DEVICE, "autotune: %s", hipGetErrorString(e));
                break;
            }
            int64_t launches = 0;
            int32_t ran = 0;
            if (t1 > 0) s = run_steps_inner(ctx, *problem, a, q, ws, 0, t1, false, st, launches, ran);
            if (s != QPA_OK) break;
            e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&took, e0, e1);
            if (e != hipSuccess) s = fail(ctx, QPA_E_DEVICE, "autotune: %s", hipGetErrorString(e));
        }
        if (s != QPA_OK) break;
        if (ms) ms[c] = took;
        if (best < 0.0 || took < best) {
            best = took;
            pick = cand[c];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != QPA_OK) return s;
    record_choice(ctx, *problem, *params, pick);
    *choice = pick;
    return QPA_OK;
}

qpa_status qpa_autotune_batch(qpa_ctx *ctx, int32_t count, const qpa_problem *problems,
                              const qpa_params *params, int32_t probe_steps, void *stream,
                              double *rates) {
    if (!ctx) return QPA_E_ARG;
    ctx->err.clear();
    qpa_status s = check_batch_params(ctx, params);
    if (s != QPA_OK) return s;
    if (probe_steps < 1) return fail(ctx, QPA_E_ARG, "probe_steps must be >= 1");
    if (count < 1 || !problems) return fail(ctx, QPA_E_ARG, "count must be >= 1, problems non-NULL");
    QPA_HIP(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    qpa_params a = *params;
    a.steps = probe_steps;
    a.lambda_table = nullptr;                 // the schedule's values do not change the cost
    const int64_t R = a.replicas;
    double measured[2] = {0.0, 0.0};
    const int32_t force[2] = {QPA_BATCH_DENSE, QPA_BATCH_SPARSE};
    const bool prof = ctx->prof;
    for (int f = 0; f < 2 && s == QPA_OK; ++f) {
        a.flags = force[f];
        BatchPlan bp;
        s = make_batch_plan(ctx, count, problems, a, bp);
        if (s != QPA_OK) break;
        // a workspace and outputs of the tuner's own for the probe solves
        const size_t obytes = align_up(sizeof(double) * (size_t)R + sizeof(int32_t));
        void *buf = nullptr;
        hipError_t e = hipMalloc(&buf, bp.total + obytes * (size_t)count);
        if (e != hipSuccess) {
            s = fail(ctx, QPA_E_DEVICE, "autotune_batch: %s", hipGetErrorString(e));
            break;
        }
        std::vector<qpa_outputs> outs(count);
        for (int32_t k = 0; k < count; ++k) {
            char *o = static_cast<char *>(buf) + bp.total + obytes * (size_t)k;
            outs[k] = qpa_outputs{};
            outs[k].energy = reinterpret_cast<double *>(o);
            outs[k].best = reinterpret_cast<int32_t *>(o + sizeof(double) * (size_t)R);
        }
        double ms = 0.0;
        int64_t launches = 0;
        const int32_t path = f == 0 ? QPA_PATH_BATCH_DENSE : QPA_PATH_BATCH_SPARSE;
        for (int rep = 0; rep < 2 && s == QPA_OK; ++rep) {      // the first run warms up
            ctx->prof = rep == 1;
            double d0 = 0.0;
            int64_t l0 = 0;
            if (rep == 1) (void)qpa_profile_read_path(ctx, QPA_PATH_ALL, &d0, &l0, 1);
            s = qpa_solve_batch(ctx, count, problems, &a, buf, bp.total, stream, outs.data());
            if (s == QPA_OK && rep == 1) {
                e = hipStreamSynchronize(st);
                if (e != hipSuccess) s = fail(ctx, QPA_E_DEVICE, "%s", hipGetErrorString(e));
                else s = qpa_profile_read_path(ctx, path, &ms, &launches, 1);
            }
        }
        ctx->prof = prof;
        // the work of the instances that took the path, over its step-kernel time
        double work = 0.0;
        for (int32_t k = 0; k < count && s == QPA_OK; ++k) {
            const int32_t pk = ctx->batch_paths[k];
            if (f == 0 && (pk == QPA_PATH_BATCH_DENSE || pk == QPA_PATH_BATCH_DENSE_I8))
                work += dense_step_work(round_up(problems[k].n, MF_BN8), R);
            if (f == 0 && pk == QPA_PATH_BATCH_SPARSE_I8)
                work += dense_step_work(round_up(problems[k].n, MF_BN8), R, problems[k].nnz);
            if (f == 1 && pk == QPA_PATH_BATCH_SPARSE)
                work += csr_step_work(problems[k].nnz, R);
        }
        (void)hipStreamSynchronize(st);
        (void)hipFree(buf);
        if (s == QPA_OK && ms > 0.0 && work > 0.0)
            measured[f] = work * (double)probe_steps / (ms / 1e3);
    }
    ctx->prof = prof;
    if (s != QPA_OK) return s;
    if (measured[0] > 0.0) ctx->batch_dense_Bps = measured[0];
    if (measured[1] > 0.0) ctx->batch_sparse_adds = measured[1];
    if (rates) {
        rates[0] = ctx->batch_dense_Bps > 0.0 ? ctx->batch_dense_Bps : DENSE_BPS_DEFAULT;
        rates[1] = ctx->batch_sparse_adds > 0.0 ? ctx->batch_sparse_adds : SPARSE_ADDS_DEFAULT;
    }
    return QPA_OK;
}

qpa_status qpa_tune_set(qpa_ctx *ctx, const qpa_problem *problem, const qpa_params *params,
                        int32_t choice) {
    if (!ctx) return QPA_E_ARG;
    ctx->err.clear();
    qpa_status s = check_problem(ctx, problem);
    if (s != QPA_OK) return s;
    s = check_params(ctx, params);
    if (s != QPA_OK) return s;
    if (problem->format != QPA_FMT_CSR)
        return fail(ctx, QPA_E_UNSUPPORTED, "kernel choices exist for sparse (CSR) problems");
    bool ok = choice == 0 ||
              ((choice == 1 || choice == 2 || choice == 4 || choice == 8) &&
               resident_ok(*problem, choice));
    if (choice == TUNE_BINNED) ok = make_plan(*problem, *params, 0, ctx->cus).bin_ok;
    if (!ok) return fail(ctx, QPA_E_ARG, "choice %d does not apply to this instance", choice);
    record_choice(ctx, *problem, *params, choice);
    return QPA_OK;
}

// ---------------------------------------------------------------- spectrum
namespace {

qpa_status check_spectrum(qpa_ctx *ctx, int64_t n, int32_t R) {
    if (n < 1) return fail(ctx, QPA_E_SHAPE, "n must be >= 1");
    if (R < 1) return fail(ctx, QPA_E_ARG, "R must be >= 1");
    if (R > SPECTRUM_MAX_R)
        return fail(ctx, QPA_E_UNSUPPORTED, "spectrum of more than %d replicas", SPECTRUM_MAX_R);
    return QPA_OK;
}

size_t spectrum_ws(int64_t n, int32_t R) {
    const size_t nw = (size_t)((n + 63) / 64);
    return align_up(sizeof(uint64_t) * nw * (size_t)R) + align_up(sizeof(uint64_t) * (size_t)R);
}

}  // namespace

qpa_status qpa_workspace_size_spectrum(qpa_ctx *ctx, int64_t n, int32_t R, size_t *bytes) {
    if (!bytes) return fail(ctx, QPA_E_ARG, "bytes is NULL");
    qpa_status s = check_spectrum(ctx, n, R);
    if (s != QPA_OK) return s;
    *bytes = spectrum_ws(n, R);
    return QPA_OK;
}

qpa_status qpa_spectrum(qpa_ctx *ctx, int64_t n, int32_t R, const int8_t *spins,
                        const double *energy, int32_t k, int32_t flags, void *workspace,
                        size_t workspace_bytes, void *stream, int8_t *out_spins,
                        double *out_energy, int32_t *out_count, int32_t *out_first,
                        int32_t *out_distinct) {
    if (!ctx) return QPA_E_ARG;
    ctx->err.clear();
    qpa_status s = check_spectrum(ctx, n, R);
    if (s != QPA_OK) return s;
    if (k < 0) return fail(ctx, QPA_E_ARG, "k must be >= 0");
    if (flags != 0 && flags != QPA_SPECTRUM_EXACT_ONLY)
        return fail(ctx, QPA_E_ARG, "flags must be 0 or QPA_SPECTRUM_EXACT_ONLY");
    if (!spins || !energy || !out_distinct || (k > 0 && (!out_energy || !out_count || !out_first)))
        return fail(ctx, QPA_E_ARG, "spins, energy, out_distinct and (k > 0) out_energy, "
                                    "out_count, out_first are required");
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % ALIGN) != 0)
        return fail(ctx, QPA_E_ARG, "workspace must be non-NULL and %zu-byte aligned", ALIGN);
    if (workspace_bytes < spectrum_ws(n, R))
        return fail(ctx, QPA_E_WORKSPACE, "workspace has %zu bytes, %zu needed", workspace_bytes,
                    spectrum_ws(n, R));
    QPA_HIP(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t nw = (size_t)((n + 63) / 64);
    uint64_t *bits = static_cast<uint64_t *>(workspace);
    uint64_t *hash = at<uint64_t>(workspace, align_up(sizeof(uint64_t) * nw * (size_t)R));
    QPA_HIP(launch_spectrum(n, R, spins, energy, k, flags == QPA_SPECTRUM_EXACT_ONLY, bits,
                            hash, out_spins, out_energy, out_count, out_first, out_distinct,
                            st));
    return QPA_OK;
}

}  // extern "C"
