// Internal declarations shared by the host and device parts of libfftt.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fftt.h"

namespace fftt {

constexpr int kTile = 4;         // voxels per tile edge: a 4x4x4 tile is one wavefront
constexpr int kTileVox = 64;
constexpr int kMaxBands = 4;
constexpr int kWavesPerBlock = 4;
constexpr int kMaxTable = 16384;
constexpr int kEntryPad = 4;      // zeroed entries after the last (look-ahead reads)
// Sine series of the detour function (at most kSeriesMax terms per band);
// device layout per band: [theta/2 per unit of the table coordinate,
// term count (int bits, a multiple of 4), 0, 0, a_1 .. a_n, zero padding].
constexpr int kSeriesMax = 64;
constexpr int kSeriesStride = 4 + kSeriesMax;

// Geometry of one transducer seen from one tile centre c (all exact in FP64
// except the two FP32 roundings, which the kernels compensate):
//   R_x(u)^2 = D0f^2 + n(u),  n(u) = cq + 2 d.u + |u|^2,  d = c - x_q,
// so R_x - D0f = n / (R_x + D0f) carries no cancellation.
struct TxConst {
    double d2x, d2y, d2z;   // 2 (c - x_q)
    double cq;              // |c - x_q|^2 - D0f^2
    float D0f;              // |c - x_q| rounded to FP32
    float Q0f;              // D0f^2 rounded to FP32
};
static_assert(sizeof(TxConst) == 40, "TxConst layout");

// The same constants in FP32 for the staged kernels' distances.  With
// millimetre tile offsets u, the terms of n = 2 (c - x_q).u + |u|^2 + cq are
// below ~1e-3 m^2, so FP32 rounding leaves an error of ~1e-10 m^2 in n and
// ~1e-9 m in delta = n / (R_x + D0f), a thousandth of a micrometre-sized
// table step; the cancelling detour R0 stays FP64-derived.
struct TxConst32 {
    float d2x, d2y, d2z, cq, D0f, Q0f;
};
static_assert(sizeof(TxConst32) == 24, "TxConst32 layout");

// One (tile, pair) incidence that survived culling.
struct Entry {
    int32_t p;              // internal pair index
    uint32_t sr;            // source | receiver << 16
    float R0hi, R0lo;       // detour D0f_s + D0f_r - L at the tile centre, hi + lo
};
static_assert(sizeof(Entry) == 16, "Entry layout");

// The staged J^T's copy of an entry (no low word of the detour).
struct Entry3 {
    int32_t p;
    uint32_t sr;
    float R0hi;
};
static_assert(sizeof(Entry3) == 12, "Entry3 layout");

struct GridGeom {
    int64_t dims[3];
    int64_t ntile[3];
    double origin[3];
    double spacing[3];
};

// Packed coordinates of an active tile: tx | ty << 21 | tz << 42.
constexpr uint64_t kTileCoordMask = (1ull << 21) - 1;

// Arguments of the apply kernels.
struct ApplyArgs {
    const int32_t* tiles;     // active tile ids [n_act]
    const uint64_t* tile_ijk; // packed tile coordinates [n_act]
    int64_t n_act;
    const int64_t* tptr;      // [n_act + 1]
    const Entry* ents;        // [nnz]
    const uint32_t* ents8;    // the staged J's copy: [nnz] (sr, R0hi bits) word pairs
    const Entry3* ents3;      // the staged J^T's copy (source-grouped or pair order)
    const int64_t* tptr3;     // its tile offsets [n_act + 1]
    const TxConst* txc;       // [n_act][n_tx]
    const TxConst32* txc32;   // the same in FP32 for the staged kernels
    int64_t n_tx;
    int64_t nnz;
    int64_t M;
    GridGeom g;
    const uint8_t* mask;      // [N]
    int nb;
    int ntab;
    float inv_dr[kMaxBands];  // (n-1)/r_max per band
    float xr[kMaxBands];      // inv_dr[b] / inv_dr[0] (staged kernels scale by band 0)
    double inv_dr64[kMaxBands];
    const void* tab;          // device table [nb][ntab] in the kernel's format
    const void* w;            // JT: [nb][M] weights C_p dT_p (internal pair order)
    const void* x;            // J: dc [N]
    void* out;                // JT: dc [N]; J: partials [nb][nnz]
    int waves_per_block;      // wavefronts per workgroup, sharing one tile (1..16)
    int n_cu;                 // compute units of the device (persistent grid size)
    int unroll;               // entries per inner-loop step (1, 2, 4)
    int split;                // 1: a workgroup shares one tile, its waves split the entries
    int stage_q;              // staged kernels: transducers per staged block (power of 2)
    int64_t nxy;              // 2D approximation: J reads dc[voxel mod nxy] (0: 3D)
};

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t alloc(size_t n) {
        if (n <= bytes && p) return hipSuccess;
        release();
        hipError_t e = hipMalloc(&p, n ? n : 1);
        if (e == hipSuccess) bytes = n;
        return e;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// ---- device-side launchers (kernels.hip) ----
hipError_t launch_txc(hipStream_t s, const int32_t* tiles, int64_t n_act, const double* tx,
                      int64_t n_tx, const GridGeom& g, TxConst* out);
hipError_t launch_cull(hipStream_t s, bool fill, const int32_t* tiles, int64_t n_act,
                       const TxConst* txc, int64_t n_tx, const int32_t* ps, const int32_t* pr,
                       const double* L, int64_t M, const GridGeom& g, double r_cut,
                       int64_t* counts, const int64_t* tptr, Entry* ents);
hipError_t launch_chunk_scan(hipStream_t s, int32_t* cnt, int64_t n_chunks, int64_t K,
                             int64_t* total);
hipError_t launch_group_count(hipStream_t s, const int64_t* tptr, const Entry* ents,
                              int64_t n_act, int64_t chunk, int64_t G, int32_t* cnt);
hipError_t launch_group_fill(hipStream_t s, const int64_t* tptr, const Entry* ents,
                             int64_t n_act, int64_t chunk, int64_t G, int32_t* cnt,
                             const int64_t* gptr, void* desc);
hipError_t launch_count_pv(hipStream_t s, const ApplyArgs& a, double r_max_all,
                           const double* L, const int32_t* ps, const int32_t* pr,
                           const double* tx, const int32_t* kptr, unsigned long long* pv_op,
                           unsigned long long* pv_eval);
hipError_t launch_weights(hipStream_t s, bool fp64, const void* dT, const int32_t* kptr,
                          const int32_t* kidx, const double* C, int64_t Mk, int64_t M, int nb,
                          void* w);
hipError_t launch_fill(hipStream_t s, bool fp64, void* p, int64_t n);
hipError_t launch_fill_value(hipStream_t s, bool fp64, void* p, int64_t n, double v);
// out[p] = sum_k in[p + k nxy], k < nz (FP64 sums in layer order)
hipError_t launch_sum_z(hipStream_t s, bool fp64, const void* in, int64_t nxy, int64_t nz,
                        void* out);
hipError_t launch_apply(hipStream_t s, fftt_precision prec, bool transpose,
                        const ApplyArgs& a);
// Table formats of the staged kernels.
enum StagedTable {
    STAB_NODE32 = 0,  // FP32 nodes h_k (4 bytes per node), cutoff by a select
    STAB_PAIR32 = 1,  // FP32 (h_k, h_{k+1} - h_k) (8 bytes per node), cutoff by the clamp
    STAB_BF16 = 2,    // packed BF16 (h_k, slope) (4 bytes per node)
    STAB_SERIES = 3,  // no table: the band's sine series (scalar loads, no LDS)
    STAB_NODE32Z = 4, // FP32 nodes with the top node stored as 0 (no select)
};
hipError_t launch_apply_staged(hipStream_t s, int tabfmt, bool transpose, const ApplyArgs& a);
// mode 1: out = sum_i |J_ij| (sensitivity coverage), mode 2: out = diag(J^T J),
// summed over bands and multiplied by wscale (a power of two), for the
// active voxels of a.out (others untouched); w: scratch [nb][M] (a.M =
// kernel pairs).
hipError_t launch_coverage(hipStream_t s, int tabfmt, int mode, const ApplyArgs& a,
                           const double* C, const int32_t* kptr, double wscale, float* w);
// LDS of a staged launch: tables plus q staged transducers (q * 512 bytes).
size_t staged_lds_bytes(int nb, int ntab, int tabfmt, int64_t q, int wpb);
// Batched point-spread functions: W ([nb][M][ldw], zeroed) and out ([n][N],
// zeroed) are filled for the n voxels given by (active tile, lane) pairs;
// col_tab is the FP32 (h, slope) table used for the weights.
// b3: contraction on BF16 matrix cores with three-way split operands (1 to
// 3 bands), else FP32 matrix cores.
hipError_t launch_psf(hipStream_t s, int tabfmt, const ApplyArgs& a, const int32_t* ptile,
                      const int32_t* plane, const double* C, const int32_t* kptr, double s2,
                      float* W, int64_t ldw, int n, float* out, const void* col_tab, bool b3);
size_t psf_lds_bytes(int nb, int ntab, int tabfmt, int64_t n_tx, bool b3);
// The PSF / Hessian contractions address a band's weights W [M][ldw] with
// 32-bit byte offsets built from 24-bit products.
inline bool psf_weights_fit(int64_t M, int64_t ldw) {
    return M * ldw < (int64_t(1) << 30) && ldw < (int64_t(1) << 22);
}
// Columns of the Hessian partials of l columns: l rounded up to a multiple
// of 8.  They are stored in blocks of 32 columns, [nb][block][nnz][width],
// width 32 but for the last block (the rest of the columns).
constexpr int hess_part_ld(int l) { return (l + 7) & ~7; }
// Slices per 64-pair group of the Hessian partial sums (red's S).
int hess_slices(int64_t Mk, int n_cu);
// Gauss-Newton Hessian of l dense vectors (1 to 3 bands, split-BF16 matrix
// cores): out [l][N] (zeroed) = sum_b J_b^T J_b Q * scale; part:
// nb * nnz * hess_part_ld(l) partials, red: [nb][S][Mk][l] FP64 with
// S = hess_slices(Mk, n_cu), W: [nb][Mk][ldw] (zeroed, ldw a multiple of 32
// >= l); Q: [l][ldq] model vectors.
hipError_t launch_hess_block(hipStream_t s, int tabfmt, const ApplyArgs& a, const float* Q,
                             int64_t ldq, int l, float* part, const int64_t* gptr,
                             const void* desc, int S, double* red, const double* C,
                             const int32_t* kptr, double scale, float* W, int64_t ldw,
                             float* out);
size_t jmb3_lds_bytes(int nb, int ntab, int tabfmt, int64_t n_tx);
// Several right-hand sides at once (1 to 3 bands, split-BF16 matrix cores).
// transpose = false: out [l][nb][M] = J Q for Q [l][ldq] model vectors, with
// part, red, S as for launch_hess_block (W unused).  transpose = true:
// out [l][N] = J^T dT for dT [l][nb][M] (in), W [nb][Mk][ldw] scratch (ldw a
// multiple of 32 >= l); out must be zeroed outside the active tiles.
hipError_t launch_rhs_batch(hipStream_t s, int tabfmt, bool transpose, const ApplyArgs& a,
                            const float* in, int64_t ldq, int l, float* part, const int64_t* gptr,
                            const void* desc, int S, double* red, const double* C,
                            const int32_t* kptr, const int32_t* kidx, int64_t M, uint32_t* W,
                            int64_t ldw, float* out);
// Copies of the entry lists for the staged J^T (Entry3 records).
// launch_pack_jt_entries: the same order.  launch_group_order: per tile,
// each kernel pair is oriented towards its endpoint with more entries in the
// tile (ties: the lower index; the kernel value is symmetric in source and
// receiver), the entries are grouped by that source, and every source's
// entries are split into whole groups of four (the grouped part, a multiple
// of eight entries) and the rest; steps of eight are interleaved evenly
// between the two kinds.  The tile's list is padded to a multiple of eight
// with entries of zero kernel value (pair 0, R0hi = 3e38).  gtptr:
// [n_act + 1] offsets with every tile's length rounded up to a multiple of
// eight.  Requires n_tx <= kGroupMaxTx.
constexpr int kGroupMaxTx = 1024;
// FP32 copy of the per-(tile, transducer) constants for the staged kernels.
hipError_t launch_pack_txc32(hipStream_t s, const TxConst* txc, int64_t n, TxConst32* out);
// The staged J reads only sr and R0hi of an entry: out [n][2] words, the
// same order as ents.
hipError_t launch_pack_j_entries(hipStream_t s, const Entry* ents, const uint8_t* bmask,
                                 int64_t n, uint32_t* out);
hipError_t launch_group_order(hipStream_t s, const int64_t* tptr, const Entry* ents,
                              const uint8_t* bmask, int64_t n_act, int n_tx,
                              const int64_t* gtptr, Entry3* gents);
hipError_t launch_pack_jt_entries(hipStream_t s, const Entry* ents, const uint8_t* bmask,
                                  int64_t n, Entry3* out);
// In both copies the source | receiver word is s | r << 14 | bands << 28
// (transducers below kCopyMaxTx); bands: bit b set when band b's kernel can
// be nonzero somewhere in the tile (launch_band_masks).
constexpr int kCopyMaxTx = 1 << 14;
// Per entry, the bands whose truncation radius exceeds the culling lower
// bound of the detour over the tile (r_cut[b] = R_max[b] + slack): bit b of
// bmask[e]; the other bands' kernel is zero over the whole tile.
hipError_t launch_band_masks(hipStream_t s, const int32_t* tiles, int64_t n_act,
                             const TxConst* txc, int64_t n_tx, const double* L,
                             const GridGeom& g, const double* r_cut, int nb,
                             const int64_t* tptr, const Entry* ents, uint8_t* bmask);
// J per-pair sum: S slices per 64-pair group (reduce_slices), FP64 scratch
// red [nb][S][Mk], then the rows of every caller pair of a group.
int reduce_slices(int64_t Mk, int n_cu);
hipError_t launch_reduce(hipStream_t s, bool fp64, const void* part, int64_t nnz,
                         const int64_t* gptr, const void* desc, const double* C,
                         const int32_t* kptr, const int32_t* kidx, int64_t Mk, int64_t M, int nb,
                         int S, double* red, void* dT);

// ---- solver building blocks (solve.hip) ----
hipError_t solver_dot(hipStream_t s, bool fp64, const void* a, const void* b, int64_t n,
                      double* part, double* sc, int slot, double scale);
hipError_t solver_axpby(hipStream_t s, bool fp64, void* y, const void* x, int64_t n, double ay,
                        int sy, double ax, int sx, const double* sc);
hipError_t solver_lin2(hipStream_t s, bool fp64, void* z, const void* x, const void* y, int64_t n,
                       double ax, double ay);
hipError_t solver_cgls_step(hipStream_t s, double* sc, double alpha_reg);
hipError_t solver_cgls_beta(hipStream_t s, double* sc);
hipError_t solver_lsqr_beta(hipStream_t s, double* sc);
hipError_t solver_lsqr_alpha_rot(hipStream_t s, double* sc, double damp, int first);
hipError_t solver_unit(hipStream_t s, bool fp64, void* x, int64_t n, int64_t v);
// Zeroes the index ranges (start, length pairs, nruns of them) of each of n
// FP32 vectors of length N.
hipError_t fill_runs(hipStream_t s, float* out, int64_t N, int n, const int64_t* runs,
                     int64_t nruns);
hipError_t solver_jacobi(hipStream_t s, bool fp64, void* minv, const float* diag, int64_t n,
                         double scale, double alpha);
hipError_t solver_mul(hipStream_t s, bool fp64, void* z, const void* a, const void* b,
                      int64_t n);

// ---- low-rank Hessian analysis (lowrank.hip) ----
// out [la][lb] (FP64) = A B^T over n rows (A: [la][n], B: [lb][n]);
// part: scratch of gram_part_doubles(la, lb, n) doubles.
hipError_t launch_gram(hipStream_t s, bool fp64, const void* A, int la, const void* B, int lb,
                       int64_t n, double* part, double* out);
size_t gram_part_doubles(int la, int lb, int64_t n);
// out [m][n] = sum_a Y[a][.] X[a][b] (X: device [l][m] FP64)
hipError_t launch_combine(hipStream_t s, bool fp64, const void* Y, int l, int64_t n,
                          const double* X, int m, void* out);
hipError_t launch_lowrank_diag(hipStream_t s, bool fp64, const void* V, int k, int64_t n,
                               const double* d, double inv_alpha, void* var, void* res);
void jacobi_eigh(std::vector<double>& A, int n, std::vector<double>& w, std::vector<double>& U);

// ---- host table builder (table.cpp) ----
int build_table_from_pulse(double c0, const double* f, int64_t nt, double dt, int64_t n,
                           double r_max, double* h_out, double* r_max_out, std::string* err);
int build_series_from_pulse(double c0, const double* f, int64_t nt, double dt, double r_max,
                            double tol, int32_t max_terms, double* a_out, int32_t* n_out,
                            double* beta_out, std::string* err);

}  // namespace fftt

struct fftt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    void* scratch = nullptr;    // device address of this device's scratch array
    std::string err;

    // geometry (host)
    bool has_geom = false;
    double c0 = 0;
    int64_t n_tx = 0, M = 0, N = 0;
    // model vectors: N values (3D), or nxy2 in-plane pixels for the 2D
    // approximation, whose prism of N = nxy2 * nz voxels is the z-quadrature
    int64_t Nm = 0, nxy2 = 0, nz2 = 0;
    std::vector<uint8_t> mask2;
    std::vector<double> tx;
    std::vector<int32_t> pairs_in;        // the caller's pairs [M][2]
    // Kernel pairs: caller pairs with identical rows of J form one group
    // (same unordered transducer pair when reciprocity is used, else the
    // same ordered pair), evaluated once.  Sorted by (source, receiver);
    // group k holds caller pairs kidx[kptr[k] .. kptr[k+1]).
    int64_t Mk = 0;
    int reciprocity = 1;
    std::vector<int32_t> ps, pr, kptr, kidx;
    std::vector<double> L, C;             // per kernel pair: length, -L dV / (2 pi c0^3)
    int blk_q = 0;                        // block size last checked for the staged layout
    bool blk_ok = false;                  // every kernel pair inside one block of blk_q
    fftt::GridGeom g{};
    double dV = 0;
    std::vector<uint8_t> mask;
    std::vector<int32_t> act_tiles;
    int64_t n_fill_runs = 0;              // voxel ranges outside every active tile

    // geometry (device)
    fftt::DevBuf d_tx, d_ps, d_pr, d_kptr, d_kidx, d_L, d_C, d_mask, d_tiles, d_tile_ijk,
        d_fill_runs;

    // kernel tables
    int nb = 0;
    int ntab = 0;
    std::vector<std::vector<double>> h;
    std::vector<double> r_max;
    std::vector<bool> band_set;
    bool tab_dirty = true;
    fftt::DevBuf d_tab32, d_tab64, d_tabbf, d_tab32n;
    // optional sine series per band (same r_max as the band's table)
    std::vector<std::vector<double>> ser_a;
    std::vector<double> ser_beta;
    bool series_ready = false;           // every band has one (uploaded)
    int eval_series = 0;                 // FP32 operators evaluate the series
    fftt::DevBuf d_series;

    // culling lists
    bool lists_ok = false;
    double lists_rcut = 0;
    int64_t nnz = 0;
    int64_t pv = 0, pv_eval = 0, lanes = 0;
    fftt::DevBuf d_txc, d_tptr, d_ents, d_gptr, d_desc;
    fftt::DevBuf d_txc32;      // FP32 copy of d_txc (staged kernels)
    int64_t n_desc = 0;
    fftt::DevBuf d_ents8;      // (sr, R0hi) of every entry, the staged J's stream
    // the staged J^T's copy of the entries: grouped by source (when every
    // staged launch covers all transducers at once, see launch_group_order;
    // tile offsets d_gtptr) or in pair order (offsets d_tptr)
    bool jt_grouped = false;
    int64_t g_nnz = 0;
    fftt::DevBuf d_gtptr, d_ents3;
    int entry_order = 1;       // build the grouped copy when it applies

    // launch shape of the operator kernels
    int waves_per_block = 16;
    int n_cu = 0;
    int unroll_jt = 4;
    int unroll_j = 4;
    int split_jt = 0, split_j = 1;
    int staged = 1;            // use the LDS-staged kernels when they fit
    int unroll_jts = 8, unroll_js = 8;
    int staged_pair_table = 0; // FP32 staged kernels: 0 node table, 1 (h, slope) pairs
    bool tab_tail_zero = false; // every band's h at r_max negligible: node table top node 0
    int staged_block_max = 0;  // cap on the staged block size (0: LDS decides)
    int psf_fp32_math = 0;     // batched PSFs: 0 split-BF16 matrix cores (1-3 bands), 1 FP32
    int hess_batched = 1;      // Hessian blocks on the matrix cores where possible
    int rhs_batched = 1;       // apply_J / apply_JT of n_rhs >= 8 batched likewise
    size_t lds_limit = 65536;

    // work buffers
    fftt::DevBuf d_w, d_part, d_red, d_solve, d_scal, d_diag;
    fftt::DevBuf d_lr, d_lr_part, d_lr_small;   // low-rank analysis: blocks, Gram scratch
    fftt::DevBuf d_z3;                          // 2D: the prism's J^T before the z sum
    fftt::DevBuf d_hb_part, d_hb_red, d_hb_w;   // batched Hessian: partials, sums, weights
    fftt::DevBuf d_psfw, d_psfd;   // batched PSF weights, (tile, lane) of each voxel

    // optional event timing of the main kernels (index: 0 J, 1 J^T, 2 reduction)
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev[4];
    size_t prof_used[4] = {0, 0, 0, 0};
    // private stream of graph solves when the caller's stream is the null
    // stream (which cannot be captured); default priority
    hipStream_t graph_stream = nullptr;
    ~fftt_ctx() {
        for (auto& v : prof_ev)
            for (auto& e : v) {
                (void)hipEventDestroy(e.first);
                (void)hipEventDestroy(e.second);
            }
        if (graph_stream) (void)hipStreamDestroy(graph_stream);
    }
};
