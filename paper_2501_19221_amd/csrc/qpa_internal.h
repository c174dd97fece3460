// Internal declarations shared by the HIP translation units of libqpa.
// Nothing here is part of the public C ABI (include/qpa.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/qpa.h"

namespace qpa {

// Validation flags written by the set-up kernels (bit mask in a device int32).
enum : int32_t {
    FLAG_ASYM = 1,        // Q or J not symmetric / Ising diagonal non-zero
    FLAG_RANGE = 2,       // integer row bound >= 2^24
    FLAG_SHAPE = 4,       // CSR row pointers / column indices inconsistent
    FLAG_UNSORTED = 8,    // CSR row columns not strictly increasing
};

// Scalars produced by canonicalisation, kept in device memory.
struct CanonScalars {
    int64_t K_i64;        // 2E = H + K for integer QUBO instances (0 for Ising)
    double K_f64;         // same for float instances
    float scale;          // 2^e of the BF16 storage
    float inv_scale;      // 2^-e
    int32_t flags;        // validation bit mask
    int32_t exp2;         // e
    double max_row;       // max_i sum_j |J_ij| + |b_i|
    double max_abs;       // max |J_ij| (i != j)
};

// Element types of the caller's arrays.
inline size_t dtype_size(int32_t dt) {
    switch (dt) {
        case QPA_I8: return 1;
        case QPA_I16: return 2;
        case QPA_I32: return 4;
        case QPA_F32: return 4;
        default: return 0;
    }
}
inline bool dtype_is_int(int32_t dt) { return dt == QPA_I8 || dt == QPA_I16 || dt == QPA_I32; }

// -------------------------------------------------------------------------------------
// Launchers (each returns hipSuccess or the first HIP error).
// -------------------------------------------------------------------------------------

// Canonicalisation of a dense problem: J_f32 (n*n, diagonal zero), b_f32 (n),
// b_i64 / b_f64 (n), per-row partials, then scalars.  Jb (npad*npad bf16) is filled when
// non-null with bf16(J / 2^e), zero padded.
// parts: scratch of 4 * CANON_PARTS doubles for the two-launch reduction of large
// instances (nullptr: one launch whatever n).
constexpr int64_t CANON_PARTS = 1024;
constexpr int64_t CANON_ROWS_PER_PART = 65536;   // one finalising launch up to this n
hipError_t launch_canon_dense(const qpa_problem &p, float *J_f32, uint16_t *Jb, int64_t npad,
                              float *b_f32, int64_t *b_i64, double *b_f64, double *row_abs,
                              double *row_max, double *row_diag, double *parts,
                              CanonScalars *sc, hipStream_t st);

// Canonicalisation of a CSR problem: b_f32 / b_i64 / b_f64, validation, scalars.
// Batched canonicalisation of integer CSR instances taking the wave-per-row pass with a
// single-stage finalisation (n <= CANON_ROWS_PER_PART): instance y of a device table in
// grid row y; the scalars are cleared, the rows processed and the scalars finalised (and
// mirrored) exactly as launch_canon_csr does.  All tasks of a launch share the coupling
// and index types; max_n bounds their n.
struct CanonTask {
    const int32_t *rp;
    const void *col;
    const void *w;
    const void *lin;
    int32_t lin_dt, is_qubo, is_int, pad_;
    int64_t n, nnz;
    float *b_f32;
    int64_t *b_i64;
    double *b_f64;
    double *row_abs, *row_max, *row_k;
    CanonScalars *sc, *mirror;
};
hipError_t launch_canon_batch(const CanonTask *tasks, int32_t ntask, qpa_dtype coupling,
                              qpa_dtype index, int64_t max_n, hipStream_t st);

// mirror (optional): a second copy of the finished scalars (one slot of a batch's array).
hipError_t launch_canon_csr(const qpa_problem &p, float *b_f32, int64_t *b_i64, double *b_f64,
                            double *row_abs, double *row_max, double *row_k, double *parts,
                            CanonScalars *sc, hipStream_t st, CanonScalars *mirror = nullptr);

// x0 / m0 from the counter RNG.  Layout: element (r, i) at x[r * ld_r + i * ld_i].
hipError_t launch_init_state(int64_t n, int64_t R, uint64_t seed, float sigma0, float *x,
                             float *m, int64_t ld_r, int64_t ld_i, int64_t Rpad, int64_t npad,
                             hipStream_t st);

// Copy a [R][n] state into / out of a strided internal layout.
hipError_t launch_copy_state(int64_t n, int64_t R, const float *src, int64_t s_ld_r,
                             int64_t s_ld_i, float *dst, int64_t d_ld_r, int64_t d_ld_i,
                             hipStream_t st);

// dst[i] = src[i] for i < n, 0 for n <= i < np.
hipError_t launch_pad_f32(int64_t n, int64_t np, const float *src, float *dst, hipStream_t st);

// spins[r*n+i] = sign(x(r,i)) (int8).
hipError_t launch_export_spins(int64_t n, int64_t R, const float *x, int64_t ld_r,
                               int64_t ld_i, int8_t *spins, hipStream_t st);

// Exact energies of int8 spins [R][n] from the caller's original couplings.
// Integer: e_i64[r] = objective (and e_f64 = (double)e_i64).  Float: e_f64 only.
// words: scratch of R * ceil(n/64) uint64 (dense problems only).
int64_t energy_partial_blocks(const qpa_problem &p);
// Integer CSR instances with many entries per row run their row scan and energies with
// one wave per row.
bool csr_rows_by_wave(const qpa_problem &p);
hipError_t launch_energy(const qpa_problem &p, const int64_t *b_i64, const double *b_f64,
                         const CanonScalars *sc, const int8_t *spins, int64_t R,
                         int64_t *e_i64, double *e_f64, double *partial, int64_t partial_len,
                         uint64_t *words, hipStream_t st);

// best[0] = lowest r with minimal energy.
hipError_t launch_argmin(int64_t R, const int64_t *e_i64, const double *e_f64, int32_t *best,
                         hipStream_t st);
// Per replica: keep the state after `t` steps when its energy is below the best so far
// (always on the first sample): its spins [R][n], energy and step.
hipError_t launch_track_best(int64_t n, int64_t R, const double *energy, const int8_t *spins,
                             int32_t t, bool first, double *best_e, int32_t *best_t,
                             int8_t *best_s, hipStream_t st);

// Batched scoring of integer CSR instances: one launch per kind for all instances of a
// table (device memory), with the results of launch_export_spins + launch_energy +
// launch_argmin (the energies are exact integers, whatever the order of their sums).
struct ScoreTask {
    const float *x;              // final state, element (r, i) at x[r * ld_r + i]
    int64_t ld_r;
    int64_t n, R;
    int64_t nblk;                // energy partial blocks, energy_bits_blocks(n)
    const int32_t *rp;           // the instance's CSR (index and weight types of the launch)
    const void *col;
    const void *w;
    const int64_t *b_i64;        // canonical integer field
    const CanonScalars *sc;
    int8_t *spins;               // [R][n] output
    double *partial;             // nblk x R
    int64_t *e_i64;              // R
    double *e_f64;               // R
    int32_t *best;               // 1
    uint64_t *words;             // scratch: R * ceil(n / 64) sign words
    int32_t is_qubo;
};
// Energies of a batched scoring table: sign words, then partial sums over blocks of
// EB_ROWS rows (nblk of a task = energy_bits_blocks(n)); n <= EBITS_MAX_N.
constexpr int EB_ROWS = 16;
constexpr int64_t EBITS_MAX_N = 4096;
int64_t energy_bits_blocks(int64_t n);
hipError_t launch_export_spins_batch(const ScoreTask *tasks, int32_t ntask, int64_t max_elems,
                                     hipStream_t st);
// All tasks of one launch share the coupling and index types; max_n and max_words bound
// the table's n and R * ceil(n / 64).
hipError_t launch_energy_bits_batch(const ScoreTask *tasks, int32_t ntask, qpa_dtype coupling,
                                    qpa_dtype index, int64_t max_n, int64_t max_words,
                                    hipStream_t st);
hipError_t launch_finalize_argmin_batch(const ScoreTask *tasks, int32_t ntask, int64_t max_R,
                                        hipStream_t st);

// ---- dense PA steps ------------------------------------------------------------------
// Small instances: couplings in LDS, all steps of a replica block in one launch.
bool dense_resident_fits(int64_t n);
hipError_t launch_dense_resident(int64_t n, int64_t R, const float *J, const float *b,
                                 float *x, float *m, float *h_last, int32_t t0, int32_t t1,
                                 const float *lam, float eta, float alpha, hipStream_t st);

// Any size: one launch per step of the FP32 tiled product shared with the SBM step (128 x
// 128 tiles, 8 x 8 sums per thread, pipelined LDS reads), fused multiply-adds in ascending
// order (exact products with s = +-1, so the same sums as the definition).  Layout
// [n][Rp], Rp = dense_fp32_rpad(R): s_cur / s_nxt float +-1, x, m, h_last.
int64_t dense_fp32_rpad(int64_t R);
hipError_t launch_dense_fp32_step(int64_t n, int64_t Rp, const float *J, const float *b,
                                  const float *s_cur, float *s_nxt, float *x, float *m,
                                  float *h_last, int32_t t, const float *lam, float eta,
                                  float alpha, hipStream_t st);
hipError_t launch_sign_f32(int64_t count, const float *x, float *s, hipStream_t st);

// BF16 matrix-core path.  Internal padded layout: x, m [Rp][np] FP32, Jb [np][np] bf16,
// spins Rp * np / 8 uint32 "pair words" (see the step kernel), chunk-major.
constexpr int MF_BM = 128;   // replicas per tile
constexpr int MF_BN = 128;   // variables per tile
constexpr int MF_NPAD = 128; // np is a multiple of this (the reduction chunk)
// Tiles of the grouped int8 step: 64 replicas x 256 variables (np a multiple of 256).
constexpr int MF_BM8 = 64, MF_BN8 = 256;
hipError_t launch_mfma_pack_spins(int64_t Rp, int64_t np, const float *x, uint32_t *sbits,
                                  hipStream_t st);
hipError_t launch_mfma_step(int64_t Rp, int64_t np, int64_t rlive, const uint16_t *Jb,
                            const float *b, const CanonScalars *sc, const uint32_t *s_cur,
                            uint32_t *s_nxt, float *x, float *m, float *h_last, int32_t t,
                            const float *lam, float eta, float alpha, hipStream_t st);
// One tile of a grouped launch (many instances, one PA step each).
struct MfmaTile {
    const uint16_t *Jb;
    const float *b;
    const CanonScalars *sc;
    uint32_t *s0, *s1;       // spin-bit buffers: step t reads s0 if t is even, else s1
    float *x, *m;            // [Rp][np] state of the instance
    const uint32_t *E;       // sparse int8 tiles: nonzero entries (see below)
    const int32_t *O;        // sparse int8 tiles: entry offsets per block, nblk + 1
    int64_t np, Rp, I0, R0, rlive;
};
// Kinds of grouped tiles: BF16 couplings; int8 couplings (integer |J| <= 127) read as
// dense rows; int8 couplings read as lists of their nonzero entries.
enum GroupKind : int { GK_BF16 = 0, GK_I8 = 1, GK_I8_SPARSE = 2 };
hipError_t launch_mfma_grouped(const MfmaTile *tiles, int32_t ntiles, int32_t t,
                               const float *lam, float eta, float alpha, GroupKind kind,
                               hipStream_t st);

// Sparse int8 tiles.  The int8 matrix J8 [np][np] is cut into blocks of 16 rows by 128
// columns, ordered (row tile of 128, column chunk of 128, row group of 16 within the row
// tile): block index ((I0 / 128) * (np / 128) + kc) * 8 + g.  Each nonzero of a block is
// one 32-bit entry: bits 0..13 its byte position in the 128 x 128 staging block of the
// step kernel (row r = I0-relative row, column k: 128 r + 16 ((k / 16) ^ (r % 8)) +
// k % 16), bits 16..23 the int8 weight.  O[blk] .. O[blk + 1] are the entries of a
// block.  A block may hold at most I8S_BLOCK_MAX entries (the step kernel prefetches that
// many per row group); denser instances keep the dense int8 rows.
constexpr int I8S_EPL = 6;                       // entries per lane of a row-group wave
constexpr int32_t I8S_BLOCK_MAX = 64 * I8S_EPL;  // entries per block of 16 x 128
__host__ __device__ inline int64_t i8s_blocks(int64_t np) { return (np / 128) * (np / 128) * 8; }
struct I8sTask {
    const int8_t *J8;        // [np][np]
    int32_t *cnt;            // nblk + 1 counts, then offsets (in place)
    uint32_t *E;             // entries
    int32_t *stats;          // [0]: largest block count, [1]: total entries
    int64_t np;
};
// count: entries of every block and the per-instance largest block and total;
// scan: counts -> offsets (exclusive, nblk + 1 values); fill: the entries.
hipError_t launch_i8s_count(const I8sTask *tasks, int32_t ntask, int64_t max_np,
                            hipStream_t st);
hipError_t launch_i8s_scan(const I8sTask *tasks, int32_t ntask, hipStream_t st);
hipError_t launch_i8s_fill(const I8sTask *tasks, int32_t ntask, int64_t max_np,
                           hipStream_t st);
// Byte spins (chunk-major, Rp * np bytes) and the int8 couplings of a CSR instance.
hipError_t launch_mfma_pack_spins_i8(int64_t Rp, int64_t np, const float *x, uint8_t *s8,
                                     hipStream_t st);
hipError_t launch_csr_to_i8(const qpa_problem &p, int64_t np, int8_t *J8, hipStream_t st);

// Batched set-up of the int8 dense slots of a batch (instance y of a device table in grid
// row y): the int8 matrix row by row (all instances of a launch share the coupling and
// index types; np at most 65536), and x0, m0, byte spins and padded field (each as the
// single-instance launchers write them).
struct SlotInitTask {
    const int32_t *rp;
    const void *col;
    const void *w;
    const float *bf;             // canonical FP32 field (n)
    int8_t *J8;                  // np x np
    float *bfp;                  // np
    float *x, *m;                // [Rp][np]
    uint8_t *s8;                 // byte spins, Rp * np
    int64_t n, np, R, Rp;
    uint64_t seed;
};
hipError_t launch_csr_to_i8_batch(const SlotInitTask *tasks, int32_t ntask, qpa_dtype coupling,
                                  qpa_dtype index, int64_t max_np, hipStream_t st);
hipError_t launch_slot_init_batch(const SlotInitTask *tasks, int32_t ntask, int64_t max_elems,
                                  float sigma0, hipStream_t st);
hipError_t launch_csr_to_bf16(const qpa_problem &p, int64_t np, const CanonScalars *sc,
                              uint16_t *Jb, hipStream_t st);

// ---- CSR PA steps --------------------------------------------------------------------
// Internal layout: x, m [np][Rp] (replica fastest, Rp a multiple of the replica group
// G), spin bits: words of 64 bits, group g, word w = bits of variables
// w*V .. w*V+V-1 (V = 64/G), G bits per variable, bit set <=> spin -1.
struct CsrView {
    int64_t n;
    const int32_t *rp;
    const void *col;
    const void *w;
    int32_t col_dt, w_dt;
    bool skip_diag;      // QUBO: diagonal entries are folded into b
    int64_t nnz = 0;
};
// Resident sparse steps: the state of G replicas x all variables stays in registers and
// the CSR structure in LDS for all steps of one launch (G in {1, 2, 4, 8}).
constexpr int64_t RES_MAX_N = 8192;
constexpr size_t RES_MAX_LDS = 160 * 1024;
size_t csr_resident_lds(int64_t n, int64_t nnz);
// G for R replicas on `cus` compute units, 0 when the instance does not fit the kernel.
int csr_resident_group(int64_t n, int64_t R, int cus);
// small_w (integer couplings only): every row's sum of |w| is below 2^16, which selects
// the packed two-replicas-per-word field sums.
hipError_t launch_csr_resident(const CsrView &c, int G, int64_t R, int64_t Rp, bool is_int,
                               bool small_w, const float *b, float *x, float *m, float *h_last,
                               int32_t t0, int32_t t1, const float *lam, float eta, float alpha,
                               hipStream_t st);
int csr_group_size(int64_t R);
int64_t csr_words_per_group(int64_t n, int G);
hipError_t launch_csr_pack_spins(int64_t n, int64_t Rp, int G, const float *x, uint64_t *sbits,
                                 hipStream_t st);
hipError_t launch_csr_step(const CsrView &c, int64_t Rp, int G, const float *b_f32,
                           const uint64_t *s_cur, uint64_t *s_nxt, float *x, float *m,
                           float *h_last, int32_t t, const float *lam, float eta, float alpha,
                           bool is_int, hipStream_t st);

// Binned sparse steps (int8 / int16 couplings, one replica group of G <= 8 lanes, the
// streamed kernel's state and spin-word layout).  Source chunks of 2^20 / G variables,
// destination bins of 2^14 L / G rows with L field sums per 32-bit LDS word (L = 1, 2 or
// 4, L <= G; every row's sum of |w| must stay below 2^(32 / L)), M = chunks x bins blocks
// of entries.
constexpr int BIN_MAX_CHUNKS = 2048;
struct BinGeom {
    int G = 0, lanes = 1, shiftG = 0, cshift = 0, bshift = 0;
    int64_t Nc = 0, Nb = 0, M = 0;
};
// Fills g; false when the instance has too many chunks or blocks for the kernels.
bool bin_geometry(int64_t n, int G, int lanes, BinGeom &g);
int64_t bin_scan_tiles(const BinGeom &g);
// Entry order of the binned kernels: off (M + 1 int32: block offsets, off[M] = entries),
// cur (M int32 scratch), tsum (bin_scan_tiles int32 scratch), src / drec (nnz uint32),
// crow (n int32: sum over the row of |w| plus the canonical integer field b_i64).
hipError_t launch_bin_build(const CsrView &c, const BinGeom &g, const int64_t *b_i64,
                            int32_t *off, int32_t *cur, int32_t *tsum, uint32_t *src,
                            uint32_t *drec, int32_t *crow, hipStream_t st);
// One PA step: s_cur -> bits (nnz bytes) -> fields, update, s_nxt.
hipError_t launch_bin_step(const BinGeom &g, int64_t n, int64_t nwords, const int32_t *off,
                           const uint32_t *src, const uint32_t *drec, uint8_t *bits,
                           const int32_t *crow, const uint64_t *s_cur, uint64_t *s_nxt, float *x,
                           float *m, float *h_last, int32_t t, const float *lam, float eta,
                           float alpha, int cus, hipStream_t st);

// ---- relaxed PA and its adjoint (FP32 state, FP64 inner products) -------------------
// Every state vector of a relaxed pass is [rows][Rp] FP32 (replica fastest); instance k
// of a batch owns global rows [row0, row0 + n).  Launch modes (see k_adjoint.hip):
enum RelModeCode : int32_t { REL_MODE_FWD = 0, REL_MODE_LOSS = 1, REL_MODE_A = 2, REL_MODE_B = 3,
                             REL_MODE_BA = 4 };
// One instance of a row launch (a CSR gather, or the element-wise pass over all rows).
struct RelInst {
    const int32_t *rp;          // CSR row pointers (NULL: no gather; dense instances)
    const void *col;
    const void *w;
    const float *b;             // canonical Ising field, n floats
    int64_t n;
    int64_t row0;               // first global row of the instance
    int64_t item0;              // first row of the instance among the launch's rows
    int64_t blk0;               // first 64-row block of the instance among the launch's
    int32_t skip_diag;          // a QUBO: stored diagonal entries are skipped
    int32_t pad_;
};
struct RelArgs {
    int64_t Rp;
    int32_t R;
    int32_t t_f;               // schedule index of the forward step (FWD) or of B (B, BA)
    int32_t t_a;               // schedule index of A (A, BA)
    int32_t nblk;              // stride of the three rows of a step's partial table
    int32_t slot0;             // first partial slot of this launch
    const float *lam;          // device schedule table
    float eta, alpha;
    double scale;
    const float *xi, *mi;      // FWD, LOSS: state of step t (xi also the product's input)
    float *xo, *mo, *fo;       // FWD: state of step t+1, f_t (fo optional)
    const float *sx, *sm, *sf; // A, BA: stored state of the A step
    const float *mu_in;        // B, BA: mu_{t+1} (product input); A: mu_{t+2} (own)
    float *mu_out;             // A, BA: mu of the A step
    float *yb;                 // A, BA: ybar written; B, BA: ybar of B read (own)
    float *xbar;               // LOSS, B: written; A: xbar_{t+1} read (own)
    double *part;              // A, BA: partial table of the A step; LOSS: loss partials
};
// Workgroups of the dense tiled product of an n-row instance.
int64_t rel_tile_blocks(int64_t n, int64_t Rp);
// Row launches over a device table of instances sharing coupling / index types (wdt, idt;
// ignored by REL_MODE_A), in blocks of 64 rows: the CSR product modes (FWD, LOSS, B, BA)
// with the product's input staged through LDS, and the element-wise REL_MODE_A over the
// rows of every instance; `blocks` = the sum of ceil(n / 64) over the table's instances;
// rel_gather_blocks = the launch's workgroups (each writes one partial slot).
constexpr int64_t REL_GATHER_BLOCKS_MAX = 512;     // two resident workgroups per CU
int64_t rel_gather_blocks(int64_t blocks, int32_t C);
hipError_t launch_rel_gather(int32_t mode, const RelInst *insts, int32_t ninst, int64_t blocks,
                             int32_t C, int32_t wdt, int32_t idt, const RelArgs &a,
                             hipStream_t st);
// Dense instance (FP32 canonical J, n x n) through the tiled product; the state pointers
// of `a` point at the instance's first row (Rp a multiple of 128).  Not REL_MODE_A.
hipError_t launch_rel_tiles(int32_t mode, int64_t n, const float *J, const float *b,
                            const RelArgs &a, hipStream_t st);
hipError_t launch_rel_fill(double *p, int64_t count, hipStream_t st);
// loss = sum of the loss partials; d_lam[t] (if non-NULL), d_eta, d_alpha from the
// per-step tables [T][3][nblk] (overwritten), all in a fixed order.
hipError_t launch_rel_finish(int32_t T, int32_t nblk, double *part_steps,
                             const double *part_loss, double *loss, double *d_eta,
                             double *d_alpha, double *d_lam, hipStream_t st);

// ---- Simulated Bifurcation Machine (App. B) -----------------------------------------
// State q, p [n][Rp] FP32 (replica fastest).  Rp: replicas padded to the dense tile (128)
// or to the CSR replica group (a power of two <= 64).
int sbm_csr_group(int64_t R);
int64_t sbm_rpad(const qpa_problem &p, int64_t R);
// One symplectic-Euler step: q_out, p from q_in, p (p in place); g_out (or NULL) receives
// the fields J q + b.  Dense problems use the canonical FP32 couplings Jf; CSR problems
// the caller's arrays (QUBO diagonal skipped).  c0 is read from device memory.
hipError_t launch_sbm_step(const qpa_problem &p, const float *Jf, int64_t Rp, const float *b,
                           const float *c0p, float a, float a0, float dt, const float *q_in,
                           float *q_out, float *pm, float *g_out, hipStream_t st);
hipError_t launch_set_f32(float *dst, float v, hipStream_t st);
// Resident CSR SBM steps (n <= RES_MAX_N): all steps in one launch, G replicas per
// workgroup; atab[t] = a(t).  0 when the instance does not fit.
int sbm_resident_group(const qpa_problem &p, int64_t R, int cus);
hipError_t launch_sbm_resident(const qpa_problem &p, int G, int64_t R, int64_t Rp,
                               const float *b, const float *c0p, const float *atab, float a0,
                               float dt, float *q, float *pm, float *g_out, int32_t t0,
                               int32_t t1, hipStream_t st);
// FP64 power method on the canonical couplings.  v, w: n doubles each; part: pw_blocks
// doubles; nrm: 2 doubles.  rho (or NULL) receives the estimate of max |lambda|, c0 (or
// NULL) the float of its reciprocal.
int64_t pw_blocks(const qpa_problem &p);
hipError_t launch_power_method(const qpa_problem &p, int32_t iters, uint64_t seed, double *v,
                               double *w, double *part, double *nrm, double *rho, float *c0,
                               hipStream_t st);

// ---- low-energy spectrum of a sample set -------------------------------------------
constexpr int32_t SPECTRUM_MAX_R = 4096;
size_t spectrum_lds_bytes(int32_t RP);
// bits: R * ceil(n/64) uint64, hash: R uint64 (workspace).
hipError_t launch_spectrum(int64_t n, int32_t R, const int8_t *spins, const double *energy,
                           int32_t k, int32_t no_hash, uint64_t *bits, uint64_t *hash,
                           int8_t *out_spins, double *out_energy, int32_t *out_count,
                           int32_t *out_first, int32_t *out_distinct, hipStream_t st);

// ---- batched CSR instances: one persistent launch ------------------------------------
struct BatchTask {
    int64_t n;
    const int32_t *rp;
    const void *col;
    const void *w;
    int32_t col_dt, w_dt;
    int32_t is_int, skip_diag;
    const float *b;          // canonical field bias b (FP32), n entries
    float *x, *m;            // [n][64] state slice of this replica group
    uint64_t seed;           // the instance's seed
    int32_t group, nrep;     // replica group index and live replicas in it (<= 64)
};
size_t batch_lds_bytes(int32_t max_n);
hipError_t launch_csr_batch(const BatchTask *tasks, int32_t ntasks, int32_t *next_task,
                            int32_t blocks, int32_t T, const float *lam, float eta, float alpha,
                            float sigma0, int32_t max_n, hipStream_t st);

}  // namespace qpa
