// C ABI entry points: context, validation, geometry pre-pass, table upload,
// and dispatch of the operator kernels.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>

#include "internal.h"

using namespace fftt;

#define FFTT_HIP(ctx, expr)                                                          \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess) {                                                     \
            (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);         \
            return e_ == hipErrorOutOfMemory ? FFTT_E_NOMEM : FFTT_E_DEVICE;        \
        }                                                                           \
    } while (0)

#define FFTT_BAD(ctx, msg)          \
    do {                            \
        (ctx)->err = (msg);         \
        return FFTT_E_INVALID;      \
    } while (0)

#define FFTT_FAIL(ctx, code, msg)   \
    do {                            \
        (ctx)->err = (msg);         \
        return (code);              \
    } while (0)

namespace {

bool finite3(const double* v) {
    return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

uint16_t bf16_rne(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

fftt_status set_device(fftt_ctx* c) {
    FFTT_HIP(c, hipSetDevice(c->device));
    return FFTT_OK;
}

double r_max_all(const fftt_ctx* c) {
    double r = 0.0;
    for (double v : c->r_max) r = std::max(r, v);
    return r;
}

fftt_status upload_tables(fftt_ctx* c) {
    if (!c->tab_dirty) return FFTT_OK;
    const int nb = c->nb, n = c->ntab;
    std::vector<float> t32((size_t)nb * n * 2);
    std::vector<double> t64((size_t)nb * n * 2);
    std::vector<uint32_t> tbf((size_t)nb * n);
    std::vector<float> tnode((size_t)nb * n + 1, 0.f);   // + h_n = 0 after the last band
    // When h at r_max is below 1e-6 of max |h| in every band (the tables of
    // build_table_from_pulse: ~1e-7), the node table stores the top node as 0
    // and the staged kernels truncate without a select; h then falls to 0
    // across the last interval instead of to h_{n-1}.  Otherwise the exact
    // nodes and the select.
    c->tab_tail_zero = n >= 2;
    for (int b = 0; b < nb; ++b) {
        double hmax = 0.0;
        for (double v : c->h[b]) hmax = std::max(hmax, std::fabs(v));
        if (!(std::fabs(c->h[b][n - 1]) <= 1e-6 * hmax)) c->tab_tail_zero = false;
    }
    for (int b = 0; b < nb; ++b) {
        const std::vector<double>& h = c->h[b];
        for (int k = 0; k < n; ++k) {
            const size_t i = (size_t)b * n + k;
            tnode[i] = (c->tab_tail_zero && k == n - 1) ? 0.f : (float)h[k];
            if (k < n - 1) {
                t64[2 * i] = h[k];
                t64[2 * i + 1] = h[k + 1] - h[k];
                t32[2 * i] = (float)h[k];
                t32[2 * i + 1] = (float)(h[k + 1] - h[k]);
                const uint16_t lo = bf16_rne((float)h[k]);
                uint32_t lo32 = (uint32_t)lo << 16;
                float lo_f;
                std::memcpy(&lo_f, &lo32, 4);
                const uint16_t hi = bf16_rne((float)(h[k + 1] - (double)lo_f));
                tbf[i] = (uint32_t)lo | ((uint32_t)hi << 16);
            } else {
                t64[2 * i] = t64[2 * i + 1] = 0.0;
                t32[2 * i] = t32[2 * i + 1] = 0.f;
                tbf[i] = 0u;
            }
        }
    }
    FFTT_HIP(c, c->d_tab32.alloc(t32.size() * sizeof(float)));
    FFTT_HIP(c, c->d_tab64.alloc(t64.size() * sizeof(double)));
    FFTT_HIP(c, c->d_tabbf.alloc(tbf.size() * sizeof(uint32_t)));
    FFTT_HIP(c, c->d_tab32n.alloc(tnode.size() * sizeof(float)));
    FFTT_HIP(c, hipMemcpy(c->d_tab32n.p, tnode.data(), tnode.size() * sizeof(float),
                          hipMemcpyHostToDevice));
    FFTT_HIP(c, hipMemcpy(c->d_tab32.p, t32.data(), t32.size() * sizeof(float),
                          hipMemcpyHostToDevice));
    FFTT_HIP(c, hipMemcpy(c->d_tab64.p, t64.data(), t64.size() * sizeof(double),
                          hipMemcpyHostToDevice));
    FFTT_HIP(c, hipMemcpy(c->d_tabbf.p, tbf.data(), tbf.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice));
    // sine series: [theta/2 per table-coordinate unit, n rounded up to a
    // multiple of 4 (int bits), 0, 0, a_1 .. a_n, zeros]
    c->series_ready = true;
    for (int b = 0; b < nb; ++b) c->series_ready = c->series_ready && !c->ser_a[b].empty();
    if (c->series_ready) {
        std::vector<float> ser((size_t)nb * kSeriesStride, 0.f);
        for (int b = 0; b < nb; ++b) {
            float* row = ser.data() + (size_t)b * kSeriesStride;
            const int32_t nt = (int32_t)c->ser_a[b].size();
            const int32_t n4 = (nt + 3) / 4 * 4;
            row[0] = (float)(0.5 * c->ser_beta[b] * c->r_max[b] / (double)(n - 1));
            std::memcpy(&row[1], &n4, sizeof(n4));
            for (int32_t m = 0; m < nt; ++m) row[4 + m] = (float)c->ser_a[b][m];
        }
        FFTT_HIP(c, c->d_series.alloc(ser.size() * sizeof(float)));
        FFTT_HIP(c, hipMemcpy(c->d_series.p, ser.data(), ser.size() * sizeof(float),
                              hipMemcpyHostToDevice));
    }
    c->tab_dirty = false;
    return FFTT_OK;
}

// Kernel pairs from the caller's pairs.  Rows of J depend on the pair only
// through R_xs + R_xr - L and L, both symmetric in source and receiver
// (source-receiver reciprocity), so with reciprocity on, (s, r) and (r, s)
// -- and repeats -- form one group evaluated once; with it off, only
// repeats of the same ordered pair are grouped.
fftt_status build_pairs(fftt_ctx* c) {
    const int64_t M = c->M;
    const int32_t* pin = c->pairs_in.data();
    auto key = [&](int64_t i) {
        const int32_t s = pin[2 * i], r = pin[2 * i + 1];
        return c->reciprocity ? std::make_pair(std::min(s, r), std::max(s, r))
                              : std::make_pair(s, r);
    };
    std::vector<int32_t> order(M);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return key(x) < key(y); });
    c->ps.clear();
    c->pr.clear();
    c->kptr.assign(1, 0);
    c->kidx = order;
    for (int64_t i = 0; i < M; ++i) {
        if (i == 0 || key(order[i]) != key(order[i - 1])) {
            c->ps.push_back(key(order[i]).first);
            c->pr.push_back(key(order[i]).second);
            if (i) c->kptr.push_back((int32_t)i);
        }
    }
    c->kptr.push_back((int32_t)M);
    const int64_t Mk = (int64_t)c->ps.size();
    c->Mk = Mk;
    c->L.resize(Mk);
    c->C.resize(Mk);
    const double c0 = c->c0;
    for (int64_t k = 0; k < Mk; ++k) {
        const double* a = c->tx.data() + 3 * c->ps[k];
        const double* b = c->tx.data() + 3 * c->pr[k];
        const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
        c->L[k] = std::sqrt(dx * dx + dy * dy + dz * dz);
        c->C[k] = -c->L[k] * c->dV / (2.0 * M_PI * c0 * c0 * c0);
    }
    FFTT_HIP(c, c->d_ps.alloc(Mk * sizeof(int32_t)));
    FFTT_HIP(c, c->d_pr.alloc(Mk * sizeof(int32_t)));
    FFTT_HIP(c, c->d_kptr.alloc((Mk + 1) * sizeof(int32_t)));
    FFTT_HIP(c, c->d_kidx.alloc(M * sizeof(int32_t)));
    FFTT_HIP(c, c->d_L.alloc(Mk * sizeof(double)));
    FFTT_HIP(c, c->d_C.alloc(Mk * sizeof(double)));
    FFTT_HIP(c, hipMemcpy(c->d_ps.p, c->ps.data(), Mk * sizeof(int32_t), hipMemcpyHostToDevice));
    FFTT_HIP(c, hipMemcpy(c->d_pr.p, c->pr.data(), Mk * sizeof(int32_t), hipMemcpyHostToDevice));
    FFTT_HIP(c, hipMemcpy(c->d_kptr.p, c->kptr.data(), (Mk + 1) * sizeof(int32_t),
                          hipMemcpyHostToDevice));
    FFTT_HIP(c, hipMemcpy(c->d_kidx.p, c->kidx.data(), M * sizeof(int32_t),
                          hipMemcpyHostToDevice));
    FFTT_HIP(c, hipMemcpy(c->d_L.p, c->L.data(), Mk * sizeof(double), hipMemcpyHostToDevice));
    FFTT_HIP(c, hipMemcpy(c->d_C.p, c->C.data(), Mk * sizeof(double), hipMemcpyHostToDevice));
    c->blk_q = 0;
    c->lists_ok = false;
    return FFTT_OK;
}

ApplyArgs base_args(const fftt_ctx* c) {
    ApplyArgs a{};
    a.tiles = c->d_tiles.as<int32_t>();
    a.tile_ijk = c->d_tile_ijk.as<uint64_t>();
    a.n_act = (int64_t)c->act_tiles.size();
    a.tptr = c->d_tptr.as<int64_t>();
    a.ents = c->d_ents.as<Entry>();
    a.ents8 = c->d_ents8.as<uint32_t>();
    a.ents3 = c->d_ents3.as<Entry3>();
    a.tptr3 = c->jt_grouped ? c->d_gtptr.as<int64_t>() : c->d_tptr.as<int64_t>();
    a.txc = c->d_txc.as<TxConst>();
    a.txc32 = c->d_txc32.as<TxConst32>();
    a.n_tx = c->n_tx;
    a.nnz = c->nnz;
    a.M = c->Mk;
    a.g = c->g;
    a.mask = c->d_mask.as<uint8_t>();
    a.nb = c->nb;
    a.ntab = c->ntab;
    a.waves_per_block = c->waves_per_block;
    a.n_cu = c->n_cu;
    a.unroll = c->unroll_jt;
    a.nxy = c->nxy2;
    for (int b = 0; b < c->nb; ++b) {
        a.inv_dr64[b] = (double)(c->ntab - 1) / c->r_max[b];
        a.inv_dr[b] = (float)a.inv_dr64[b];
        a.xr[b] = (float)(a.inv_dr64[b] / a.inv_dr64[0]);
    }
    return a;
}

fftt_status build_lists(fftt_ctx* c) {
    const int64_t n_act = (int64_t)c->act_tiles.size();
    const int64_t n_tx = c->n_tx, M = c->Mk;
    const double r_cut = r_max_all(c) + 1e-7;
    hipStream_t s = c->stream;
    c->lists_ok = false;

    FFTT_HIP(c, c->d_txc.alloc((size_t)n_act * n_tx * sizeof(TxConst)));
    FFTT_HIP(c, launch_txc(s, c->d_tiles.as<int32_t>(), n_act, c->d_tx.as<double>(), n_tx, c->g,
                           c->d_txc.as<TxConst>()));
    FFTT_HIP(c, c->d_txc32.alloc((size_t)n_act * n_tx * sizeof(TxConst32)));
    FFTT_HIP(c, launch_pack_txc32(s, c->d_txc.as<TxConst>(), n_act * n_tx,
                                  c->d_txc32.as<TxConst32>()));

    DevBuf counts;
    FFTT_HIP(c, counts.alloc((size_t)std::max<int64_t>(n_act, 1) * sizeof(int64_t)));
    FFTT_HIP(c, launch_cull(s, false, c->d_tiles.as<int32_t>(), n_act, c->d_txc.as<TxConst>(),
                            n_tx, c->d_ps.as<int32_t>(), c->d_pr.as<int32_t>(),
                            c->d_L.as<double>(), M, c->g, r_cut, counts.as<int64_t>(), nullptr,
                            nullptr));
    std::vector<int64_t> cnt(n_act), tptr(n_act + 1, 0);
    if (n_act)
        FFTT_HIP(c, hipMemcpyAsync(cnt.data(), counts.p, n_act * sizeof(int64_t),
                                   hipMemcpyDeviceToHost, s));
    FFTT_HIP(c, hipStreamSynchronize(s));
    for (int64_t a = 0; a < n_act; ++a) tptr[a + 1] = tptr[a] + cnt[a];
    const int64_t nnz = tptr[n_act];
    FFTT_HIP(c, c->d_tptr.alloc((n_act + 1) * sizeof(int64_t)));
    FFTT_HIP(c, hipMemcpyAsync(c->d_tptr.p, tptr.data(), (n_act + 1) * sizeof(int64_t),
                               hipMemcpyHostToDevice, s));
    // kEntryPad zeroed entries past the end (pair 0, transducer 0): the
    // operator kernels read one step ahead of the entry they evaluate
    FFTT_HIP(c, c->d_ents.alloc((size_t)(nnz + kEntryPad) * sizeof(Entry)));
    FFTT_HIP(c, hipMemsetAsync(c->d_ents.as<Entry>() + nnz, 0, kEntryPad * sizeof(Entry), s));
    FFTT_HIP(c, launch_cull(s, true, c->d_tiles.as<int32_t>(), n_act, c->d_txc.as<TxConst>(),
                            n_tx, c->d_ps.as<int32_t>(), c->d_pr.as<int32_t>(),
                            c->d_L.as<double>(), M, c->g, r_cut, nullptr,
                            c->d_tptr.as<int64_t>(), c->d_ents.as<Entry>()));

    // per entry, the bands whose kernel can be nonzero in the tile (carried
    // by the staged copies below)
    DevBuf bmask;
    FFTT_HIP(c, bmask.alloc((size_t)std::max<int64_t>(nnz, 1)));
    {
        double cuts[kMaxBands];
        for (int b = 0; b < c->nb; ++b) cuts[b] = c->r_max[b] + 1e-7;
        FFTT_HIP(c, launch_band_masks(s, c->d_tiles.as<int32_t>(), n_act, c->d_txc.as<TxConst>(),
                                      n_tx, c->d_L.as<double>(), c->g, cuts, c->nb,
                                      c->d_tptr.as<int64_t>(), c->d_ents.as<Entry>(),
                                      bmask.as<uint8_t>()));
    }
    // the staged J's eight-byte copy (with the same look-ahead padding)
    FFTT_HIP(c, c->d_ents8.alloc((size_t)(nnz + kEntryPad) * 2 * sizeof(uint32_t)));
    FFTT_HIP(c, hipMemsetAsync(c->d_ents8.as<uint32_t>() + 2 * nnz, 0,
                               kEntryPad * 2 * sizeof(uint32_t), s));
    FFTT_HIP(c, launch_pack_j_entries(s, c->d_ents.as<Entry>(), bmask.as<uint8_t>(), nnz,
                                      c->d_ents8.as<uint32_t>()));

    // run descriptors of 64-pair groups (for the deterministic J reduction)
    const int64_t chunk = 256;
    const int64_t n_chunks = (n_act + chunk - 1) / chunk;
    const int64_t G = (M + 63) / 64;
    DevBuf ccnt, total;
    FFTT_HIP(c, ccnt.alloc((size_t)std::max<int64_t>(n_chunks * G, 1) * sizeof(int32_t)));
    FFTT_HIP(c, total.alloc((size_t)G * sizeof(int64_t)));
    FFTT_HIP(c, hipMemsetAsync(ccnt.p, 0, (size_t)n_chunks * G * sizeof(int32_t), s));
    FFTT_HIP(c, launch_group_count(s, c->d_tptr.as<int64_t>(), c->d_ents.as<Entry>(), n_act,
                                   chunk, G, ccnt.as<int32_t>()));
    FFTT_HIP(c, launch_chunk_scan(s, ccnt.as<int32_t>(), n_chunks, G, total.as<int64_t>()));
    std::vector<int64_t> tot(G), gptr(G + 1, 0);
    FFTT_HIP(c, hipMemcpyAsync(tot.data(), total.p, G * sizeof(int64_t), hipMemcpyDeviceToHost,
                               s));
    FFTT_HIP(c, hipStreamSynchronize(s));
    for (int64_t g = 0; g < G; ++g) gptr[g + 1] = gptr[g] + tot[g];
    c->n_desc = gptr[G];
    FFTT_HIP(c, c->d_gptr.alloc((G + 1) * sizeof(int64_t)));
    FFTT_HIP(c, hipMemcpyAsync(c->d_gptr.p, gptr.data(), (G + 1) * sizeof(int64_t),
                               hipMemcpyHostToDevice, s));
    FFTT_HIP(c, c->d_desc.alloc((size_t)std::max<int64_t>(c->n_desc, 1) * 16));
    FFTT_HIP(c, launch_group_fill(s, c->d_tptr.as<int64_t>(), c->d_ents.as<Entry>(), n_act,
                                  chunk, G, ccnt.as<int32_t>(), c->d_gptr.as<int64_t>(),
                                  c->d_desc.p));
    c->nnz = nnz;

    // exact work counts (FP64 decision R < R_max): over caller pairs and
    // over the evaluated kernel pairs
    DevBuf pvb;
    FFTT_HIP(c, pvb.alloc(2 * sizeof(unsigned long long)));
    FFTT_HIP(c, hipMemsetAsync(pvb.p, 0, 2 * sizeof(unsigned long long), s));
    ApplyArgs a = base_args(c);
    FFTT_HIP(c, launch_count_pv(s, a, r_max_all(c), c->d_L.as<double>(), c->d_ps.as<int32_t>(),
                                c->d_pr.as<int32_t>(), c->d_tx.as<double>(),
                                c->d_kptr.as<int32_t>(), pvb.as<unsigned long long>(),
                                pvb.as<unsigned long long>() + 1));
    unsigned long long pv[2] = {0, 0};
    FFTT_HIP(c, hipMemcpyAsync(pv, pvb.p, sizeof(pv), hipMemcpyDeviceToHost, s));
    FFTT_HIP(c, hipStreamSynchronize(s));
    c->pv = (int64_t)pv[0];
    c->pv_eval = (int64_t)pv[1];
    c->lanes = nnz * kTileVox;

    // the staged J^T's twelve-byte copy: grouped by source when every staged
    // launch stages all transducers at once (the tables in their largest
    // layout plus 512 bytes per transducer fit in LDS), else in pair order
    c->jt_grouped = false;
    c->d_gtptr.release();
    const bool one_block = n_tx <= kGroupMaxTx &&
                           staged_lds_bytes(c->nb, c->ntab, STAB_PAIR32, n_tx,
                                            c->waves_per_block) <= c->lds_limit;
    if (c->entry_order && one_block) {
        std::vector<int64_t> gt(n_act + 1, 0);
        for (int64_t a = 0; a < n_act; ++a) gt[a + 1] = gt[a] + (cnt[a] + 7) / 8 * 8;
        c->g_nnz = gt[n_act];
        FFTT_HIP(c, c->d_gtptr.alloc((n_act + 1) * sizeof(int64_t)));
        FFTT_HIP(c, hipMemcpyAsync(c->d_gtptr.p, gt.data(), (n_act + 1) * sizeof(int64_t),
                                   hipMemcpyHostToDevice, s));
        FFTT_HIP(c, c->d_ents3.alloc((size_t)(c->g_nnz + kEntryPad) * sizeof(Entry3)));
        FFTT_HIP(c, hipMemsetAsync(c->d_ents3.as<Entry3>() + c->g_nnz, 0,
                                   kEntryPad * sizeof(Entry3), s));
        FFTT_HIP(c, launch_group_order(s, c->d_tptr.as<int64_t>(), c->d_ents.as<Entry>(),
                                       bmask.as<uint8_t>(), n_act, (int)n_tx,
                                       c->d_gtptr.as<int64_t>(), c->d_ents3.as<Entry3>()));
        // the host offsets must outlive the asynchronous copy
        FFTT_HIP(c, hipStreamSynchronize(s));
        c->jt_grouped = true;
    } else {
        FFTT_HIP(c, c->d_ents3.alloc((size_t)(nnz + kEntryPad) * sizeof(Entry3)));
        FFTT_HIP(c, hipMemsetAsync(c->d_ents3.as<Entry3>() + nnz, 0, kEntryPad * sizeof(Entry3),
                                   s));
        FFTT_HIP(c, launch_pack_jt_entries(s, c->d_ents.as<Entry>(), bmask.as<uint8_t>(), nnz,
                                           c->d_ents3.as<Entry3>()));
    }
    c->lists_rcut = r_cut;
    c->lists_ok = true;
    return FFTT_OK;
}



// Event pair for one timed launch of kernel family k (or nulls when off).
hipError_t prof_begin(fftt_ctx* c, int k, hipEvent_t* stop) {
    *stop = nullptr;
    if (!c->prof) return hipSuccess;
    auto& v = c->prof_ev[k];
    if (c->prof_used[k] == v.size()) {
        hipEvent_t a, b;
        hipError_t e = hipEventCreate(&a);
        if (e != hipSuccess) return e;
        e = hipEventCreate(&b);
        if (e != hipSuccess) return e;
        v.emplace_back(a, b);
    }
    auto& ev = v[c->prof_used[k]++];
    *stop = ev.second;
    return hipEventRecord(ev.first, c->stream);
}

hipError_t prof_end(fftt_ctx* c, hipEvent_t stop) {
    return stop ? hipEventRecord(stop, c->stream) : hipSuccess;
}

// Table format of the LDS-staged kernels for an FP32 / BF16-table apply.
int staged_table(const fftt_ctx* c, fftt_precision prec) {
    if (prec == FFTT_FP32_BF16TABLE) return STAB_BF16;
    if (c->staged_pair_table) return STAB_PAIR32;
    return c->tab_tail_zero ? STAB_NODE32Z : STAB_NODE32;
}

// Evaluation of the detour function by the J / J^T kernels: the staged
// table, or for FP32 with FFTT_TUNE_KERNEL_EVAL the sine series.
int op_table(const fftt_ctx* c, fftt_precision prec) {
    return (prec == FFTT_FP32 && c->eval_series) ? STAB_SERIES : staged_table(c, prec);
}

// Transducers per staged block for an FP32 / BF16-table apply: the
// smallest power of two covering all transducers, halved until the tables
// plus one float2 per (transducer, lane) of the block fit in LDS; 0 when
// staging is off, nothing fits, or a kernel pair spans two blocks (the
// per-wavefront kernels run then).
int staged_q(fftt_ctx* c, fftt_precision prec) {
    // the staged kernels read the entry copies, whose transducer fields hold
    // indices below kCopyMaxTx
    if (!c->staged || prec == FFTT_FP64 || c->n_tx >= kCopyMaxTx) return 0;
    const int fmt = op_table(c, prec);
    int q = 16;
    while (q < c->n_tx) q *= 2;
    while (q >= 16 && ((c->staged_block_max && q > c->staged_block_max) ||
                       staged_lds_bytes(c->nb, c->ntab, fmt, q, c->waves_per_block) >
                           c->lds_limit))
        q /= 2;
    if (q < 16) return 0;
    if (q >= c->n_tx) return q;
    if (c->blk_q != q) {
        c->blk_q = q;
        c->blk_ok = true;
        for (int64_t k = 0; k < c->Mk && c->blk_ok; ++k)
            c->blk_ok = c->ps[k] / q == c->pr[k] / q;
    }
    return c->blk_ok ? q : 0;
}

// Device table of a staged launch.
const void* staged_table_ptr(const fftt_ctx* c, int fmt) {
    switch (fmt) {
        case STAB_NODE32:
        case STAB_NODE32Z: return c->d_tab32n.p;
        case STAB_PAIR32: return c->d_tab32.p;
        case STAB_SERIES: return c->d_series.p;
        default: return c->d_tabbf.p;
    }
}

// Batched PSFs (FP32 / BF16 table): every voxel's J^T weights, then one
// launch of the matrix-core kernel over all active tiles.
fftt_status psf_batched(fftt_ctx* c, fftt_precision prec, const int64_t* voxels, int32_t n,
                        double s2, float* out) {
    const int64_t nx = c->g.dims[0], ny = c->g.dims[1];
    std::vector<int32_t> desc(2 * (size_t)n);
    for (int32_t k = 0; k < n; ++k) {
        const int64_t v = voxels[k];
        const int64_t x = v % nx, y = (v / nx) % ny, z = v / (nx * ny);
        const int64_t t = x / kTile + c->g.ntile[0] * (y / kTile + c->g.ntile[1] * (z / kTile));
        const auto it = std::lower_bound(c->act_tiles.begin(), c->act_tiles.end(), (int32_t)t);
        if (it == c->act_tiles.end() || *it != t) FFTT_BAD(c, "psf: voxel outside active tiles");
        desc[k] = (int32_t)(it - c->act_tiles.begin());
        desc[n + k] = (int32_t)((x % kTile) + kTile * ((y % kTile) + kTile * (z % kTile)));
    }
    const int64_t ldw = ((int64_t)n + 31) / 32 * 32;
    if (!psf_weights_fit(c->Mk, ldw))
        FFTT_BAD(c, "psf: too many PSFs in one call (kernel pairs x n must stay below 2^30)");
    FFTT_HIP(c, c->d_psfd.alloc(desc.size() * sizeof(int32_t)));
    FFTT_HIP(c, hipMemcpyAsync(c->d_psfd.p, desc.data(), desc.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, c->stream));
    FFTT_HIP(c, c->d_psfw.alloc((size_t)c->nb * c->Mk * ldw * sizeof(float)));
    FFTT_HIP(c, launch_fill(c->stream, false, c->d_psfw.p, (int64_t)c->nb * c->Mk * ldw));
    FFTT_HIP(c, fill_runs(c->stream, out, c->N, n, c->d_fill_runs.as<int64_t>(),
                          c->n_fill_runs));
    ApplyArgs a = base_args(c);
    const int fmt = staged_table(c, prec);
    a.tab = staged_table_ptr(c, fmt);
    a.stage_q = (int)c->n_tx;             // one block: every transducer staged
    const void* col_tab = c->d_tab32.p;   // FP32 (h, slope) pairs
    hipEvent_t stop;
    FFTT_HIP(c, prof_begin(c, 3, &stop));
    FFTT_HIP(c, launch_psf(c->stream, fmt, a, c->d_psfd.as<int32_t>(),
                           c->d_psfd.as<int32_t>() + n, c->d_C.as<double>(),
                           c->d_kptr.as<int32_t>(), s2,
                           c->d_psfw.as<float>(), ldw, n, out, col_tab, c->psf_fp32_math == 0));
    FFTT_HIP(c, prof_end(c, stop));
    // the host descriptor buffer must outlive the asynchronous copy
    FFTT_HIP(c, hipStreamSynchronize(c->stream));
    return FFTT_OK;
}

// dT [B][M] = J dc (caller order), one right-hand side; ensure_ready done.
fftt_status apply_J_one(fftt_ctx* c, fftt_precision prec, const void* x, void* y) {
    const bool fp64 = prec == FFTT_FP64;
    const size_t es = fp64 ? sizeof(double) : sizeof(float);
    FFTT_HIP(c, c->d_part.alloc((size_t)c->nb * std::max<int64_t>(c->nnz, 1) * es));
    ApplyArgs a = base_args(c);
    a.tab = fp64 ? c->d_tab64.p : (prec == FFTT_FP32 ? c->d_tab32.p : c->d_tabbf.p);
    a.out = c->d_part.p;
    a.unroll = c->unroll_j;
    a.split = c->split_j;
    a.x = x;
    if (op_table(c, prec) == STAB_SERIES && !c->series_ready)
        FFTT_FAIL(c, FFTT_E_STATE, "series evaluation: a band has no sine series");
    hipEvent_t stop;
    FFTT_HIP(c, prof_begin(c, 0, &stop));
    if (const int q = staged_q(c, prec)) {
        a.stage_q = q;
        a.unroll = c->unroll_js;
        const int fmt = op_table(c, prec);
        a.tab = staged_table_ptr(c, fmt);
        FFTT_HIP(c, launch_apply_staged(c->stream, fmt, false, a));
    } else {
        if (op_table(c, prec) == STAB_SERIES)
            FFTT_FAIL(c, FFTT_E_UNSUPPORTED,
                      "series evaluation needs the staged kernels (FFTT_TUNE_STAGED, LDS)");
        FFTT_HIP(c, launch_apply(c->stream, prec, false, a));
    }
    FFTT_HIP(c, prof_end(c, stop));
    FFTT_HIP(c, prof_begin(c, 2, &stop));
    const int S = reduce_slices(c->Mk, c->n_cu);
    FFTT_HIP(c, c->d_red.alloc((size_t)c->nb * S * std::max<int64_t>(c->Mk, 1) * sizeof(double)));
    FFTT_HIP(c, launch_reduce(c->stream, fp64, c->d_part.p, c->nnz, c->d_gptr.as<int64_t>(),
                              c->d_desc.p, c->d_C.as<double>(), c->d_kptr.as<int32_t>(),
                              c->d_kidx.as<int32_t>(), c->Mk, c->M, c->nb, S,
                              c->d_red.as<double>(), y));
    FFTT_HIP(c, prof_end(c, stop));
    return FFTT_OK;
}

// dc [N] = J^T dT, one right-hand side, with the caller's work buffers:
// wbuf [nb][Mk] weights in the precision's type and, in the 2D mode, zbuf
// [N] for the prism's output before the layer sum.  Allocates nothing and,
// with timed = false, creates no events.  ensure_ready done.
fftt_status apply_JT_work(fftt_ctx* c, fftt_precision prec, const void* y, void* x, void* wbuf,
                          void* zbuf, bool timed) {
    const bool fp64 = prec == FFTT_FP64;
    ApplyArgs a = base_args(c);
    a.tab = fp64 ? c->d_tab64.p : (prec == FFTT_FP32 ? c->d_tab32.p : c->d_tabbf.p);
    a.w = wbuf;
    // 2D approximation: the prism's J^T first, then the sum over its layers
    void* out = c->nxy2 ? zbuf : x;
    a.out = out;
    if (op_table(c, prec) == STAB_SERIES && !c->series_ready)
        FFTT_FAIL(c, FFTT_E_STATE, "series evaluation: a band has no sine series");
    FFTT_HIP(c, launch_weights(c->stream, fp64, y, c->d_kptr.as<int32_t>(),
                               c->d_kidx.as<int32_t>(), c->d_C.as<double>(), c->Mk, c->M, c->nb,
                               wbuf));
    FFTT_HIP(c, launch_fill(c->stream, fp64, out, c->N));
    hipEvent_t stop = nullptr;
    if (timed) FFTT_HIP(c, prof_begin(c, 1, &stop));
    // the grouped copy serves launches that stage every transducer at once
    int q = staged_q(c, prec);
    if (c->jt_grouped && q < c->n_tx) q = 0;
    if (q) {
        a.stage_q = q;
        a.unroll = c->unroll_jts;
        const int fmt = op_table(c, prec);
        a.tab = staged_table_ptr(c, fmt);
        FFTT_HIP(c, launch_apply_staged(c->stream, fmt, true, a));
    } else {
        if (op_table(c, prec) == STAB_SERIES)
            FFTT_FAIL(c, FFTT_E_UNSUPPORTED,
                      "series evaluation needs the staged kernels (FFTT_TUNE_STAGED, LDS)");
        FFTT_HIP(c, launch_apply(c->stream, prec, true, a));
    }
    FFTT_HIP(c, prof_end(c, stop));
    if (c->nxy2) FFTT_HIP(c, launch_sum_z(c->stream, fp64, out, c->nxy2, c->nz2, x));
    return FFTT_OK;
}

// dc [N] = J^T dT, one right-hand side, work buffers owned by the context;
// ensure_ready done.
fftt_status apply_JT_one(fftt_ctx* c, fftt_precision prec, const void* y, void* x) {
    const size_t es = prec == FFTT_FP64 ? sizeof(double) : sizeof(float);
    FFTT_HIP(c, c->d_w.alloc((size_t)c->nb * c->Mk * es));
    if (c->nxy2) FFTT_HIP(c, c->d_z3.alloc((size_t)c->N * es));
    return apply_JT_work(c, prec, y, x, c->d_w.p, c->nxy2 ? c->d_z3.p : nullptr, true);
}

// out [N] FP32 = coverage (kind 0) or diag(J^T J) (kind 1); ensure_ready done.
fftt_status coverage_one(fftt_ctx* c, fftt_precision prec, int32_t kind, float* out) {
    if (c->nxy2)   // abs() and squares do not commute with the sum over the layers
        FFTT_FAIL(c, FFTT_E_UNSUPPORTED, "coverage / diag(J^T J) of the 2D approximation");
    const int q = staged_q(c, prec);
    if (!q)
        FFTT_FAIL(c, FFTT_E_UNSUPPORTED, "coverage needs the staged kernels (FFTT_TUNE_STAGED, LDS)");
    const int fmt = op_table(c, prec);
    if (fmt == STAB_SERIES && !c->series_ready)
        FFTT_FAIL(c, FFTT_E_STATE, "series evaluation: a band has no sine series");
    FFTT_HIP(c, c->d_w.alloc((size_t)c->nb * c->Mk * sizeof(double)));
    ApplyArgs a = base_args(c);
    a.stage_q = q;
    a.tab = staged_table_ptr(c, fmt);
    a.out = out;
    // the largest weight (|C_p| m_p or C_p^2 m_p) is scaled into [1, 2) by a
    // power of two, undone on the output (both exact)
    double wmax = 0.0;
    for (int64_t k = 0; k < c->Mk; ++k) {
        const double m = (double)(c->kptr[k + 1] - c->kptr[k]);
        wmax = std::max(wmax, kind == 0 ? std::fabs(c->C[k]) * m : c->C[k] * c->C[k] * m);
    }
    const int e = wmax > 0.0 ? std::ilogb(wmax) : 0;
    FFTT_HIP(c, launch_fill(c->stream, false, out, c->N));
    FFTT_HIP(c, launch_coverage(c->stream, fmt, kind + 1, a, c->d_C.as<double>(),
                                c->d_kptr.as<int32_t>(), std::ldexp(1.0, -e),
                                c->d_w.as<float>()));
    FFTT_HIP(c, solver_lin2(c->stream, false, out, out, nullptr, c->N, std::ldexp(1.0, e), 0.0));
    return FFTT_OK;
}

fftt_status ensure_ready(fftt_ctx* c) {
    if (!c->has_geom) {
        c->err = "geometry not set";
        return FFTT_E_STATE;
    }
    if (c->nb == 0) {
        c->err = "no kernel table set";
        return FFTT_E_STATE;
    }
    for (int b = 0; b < c->nb; ++b)
        if (!c->band_set[b]) {
            c->err = "kernel table of band " + std::to_string(b) + " missing";
            return FFTT_E_STATE;
        }
    fftt_status st = set_device(c);
    if (st != FFTT_OK) return st;
    st = upload_tables(c);
    if (st != FFTT_OK) return st;
    if (!c->lists_ok) return build_lists(c);
    return FFTT_OK;
}

// BF16 tables are not offered in the 2D approximation (eq. forward_2D): the
// z integral sums Fresnel zones of alternating sign, so the per-layer
// rounding of a BF16 table is not averaged away and J^T of sign-random data
// comes out near the 1e-3 bound of that precision.
fftt_status check_plane_precision(fftt_ctx* c, fftt_precision prec) {
    if (c->nxy2 && prec == FFTT_FP32_BF16TABLE)
        FFTT_FAIL(c, FFTT_E_UNSUPPORTED,
                  "the 2D approximation takes FFTT_FP64 or FFTT_FP32, not BF16 tables");
    return FFTT_OK;
}

// ---- randomized eigensolver for H = J^T J / sigma^2 (Sec. II-D) ----

// y = H x = J^T (J x) / sigma^2; dT: scratch [nb][M].
// Columns per batch of the multi-vector J (transpose = false) or J^T on the
// matrix cores for r right-hand sides, or 0 where the batched kernels do
// not apply (FP64, series evaluation, four bands, the 2D mode, no staged
// kernels, LDS, fewer than kRhsBatchMin vectors): the partials of J take
// nb * nnz floats per column, kept under 8 GB per batch.
constexpr int kRhsBatchMin = 8;

int rhs_batch_cols(fftt_ctx* c, fftt_precision prec, bool transpose, int r) {
    if (!c->rhs_batched || r < kRhsBatchMin || prec == FFTT_FP64 || c->nb > 3 || c->nxy2 ||
        !c->staged || op_table(c, prec) == STAB_SERIES || c->nnz == 0)
        return 0;
    const int fmt = staged_table(c, prec);
    if (psf_lds_bytes(c->nb, c->ntab, fmt, c->n_tx, true) > c->lds_limit) return 0;
    if (!transpose && jmb3_lds_bytes(c->nb, c->ntab, fmt, c->n_tx) > c->lds_limit) return 0;
    int cb = r;
    if (!transpose) {
        const double per_col = (double)c->nb * (double)c->nnz * sizeof(float);
        cb = (int)std::min<double>(r, std::floor(8e9 / per_col));
        if (cb < r) cb &= ~7;
    }
    while (cb >= kRhsBatchMin && !psf_weights_fit(c->Mk, ((int64_t)cb + 31) / 32 * 32)) cb /= 2;
    return cb >= kRhsBatchMin ? cb : 0;
}

// dT [r][nb][M] = J dc or dc [r][N] = J^T dT for r right-hand sides in
// batches of cb columns on the matrix cores; ensure_ready done.
fftt_status apply_rhs_batched(fftt_ctx* c, fftt_precision prec, bool transpose, const void* in,
                              void* out, int r, int cb) {
    const int fmt = staged_table(c, prec);
    const int64_t N = c->Nm, D = (int64_t)c->nb * c->M;
    const int S = hess_slices(c->Mk, c->n_cu);
    ApplyArgs a = base_args(c);
    a.tab = staged_table_ptr(c, fmt);
    a.stage_q = (int)c->n_tx;
    hipEvent_t stop;
    FFTT_HIP(c, prof_begin(c, transpose ? 1 : 0, &stop));
    for (int c0 = 0; c0 < r; c0 += cb) {
        const int n = std::min(cb, r - c0);
        const int64_t ldw = ((int64_t)n + 31) / 32 * 32;
        if (transpose) {
            FFTT_HIP(c, c->d_hb_w.alloc((size_t)c->nb * c->Mk * ldw * sizeof(uint32_t)));
            FFTT_HIP(c, launch_fill(c->stream, false, c->d_hb_w.p, (int64_t)c->nb * c->Mk * ldw));
            float* o = static_cast<float*>(out) + (size_t)c0 * N;
            FFTT_HIP(c, fill_runs(c->stream, o, c->N, n, c->d_fill_runs.as<int64_t>(),
                                  c->n_fill_runs));
            FFTT_HIP(c, launch_rhs_batch(c->stream, fmt, true, a,
                                         static_cast<const float*>(in) + (size_t)c0 * D, 0, n,
                                         nullptr, c->d_gptr.as<int64_t>(), c->d_desc.p, S,
                                         nullptr, c->d_C.as<double>(), c->d_kptr.as<int32_t>(),
                                         c->d_kidx.as<int32_t>(), c->M,
                                         c->d_hb_w.as<uint32_t>(), ldw, o));
        } else {
            FFTT_HIP(c, c->d_hb_part.alloc((size_t)c->nb * c->nnz * hess_part_ld(n) * sizeof(float)));
            FFTT_HIP(c, c->d_hb_red.alloc((size_t)c->nb * S * c->Mk * n * sizeof(double)));
            FFTT_HIP(c, launch_rhs_batch(c->stream, fmt, false, a,
                                         static_cast<const float*>(in) + (size_t)c0 * N, N, n,
                                         c->d_hb_part.as<float>(), c->d_gptr.as<int64_t>(),
                                         c->d_desc.p, S, c->d_hb_red.as<double>(),
                                         c->d_C.as<double>(), c->d_kptr.as<int32_t>(),
                                         c->d_kidx.as<int32_t>(), c->M, nullptr, 0,
                                         static_cast<float*>(out) + (size_t)c0 * D));
        }
    }
    FFTT_HIP(c, prof_end(c, stop));
    return FFTT_OK;
}

fftt_status hess_apply(fftt_ctx* c, fftt_precision prec, double isg2, const void* x, void* dT,
                       void* y) {
    fftt_status st = apply_J_one(c, prec, x, dT);
    if (st != FFTT_OK) return st;
    FFTT_HIP(c, solver_lin2(c->stream, prec == FFTT_FP64, dT, dT, nullptr, (int64_t)c->nb * c->M,
                            isg2, 0.0));
    return apply_JT_one(c, prec, dT, y);
}

// Y [r][Nm] = H X for r vectors: batched on the matrix cores (split BF16)
// for FP32 / BF16-table operators with 1 to 3 bands in 3D when the staged
// layouts fit LDS, in column batches whose partials stay below 8 GB; one
// vector at a time otherwise.
fftt_status hess_block(fftt_ctx* c, fftt_precision prec, double isg2, const void* X, void* Y,
                       int r, void* dT) {
    const bool fp64 = prec == FFTT_FP64;
    const size_t es = fp64 ? sizeof(double) : sizeof(float);
    const int64_t N = c->Nm;
    const int fmt = staged_table(c, prec);
    const double budget = 8e9;
    int cb = 0;
    if (c->hess_batched && !fp64 && c->nb <= 3 && !c->nxy2 && c->staged &&
        op_table(c, prec) != STAB_SERIES &&
        jmb3_lds_bytes(c->nb, c->ntab, fmt, c->n_tx) <= c->lds_limit &&
        psf_lds_bytes(c->nb, c->ntab, fmt, c->n_tx, true) <= c->lds_limit && c->nnz > 0) {
        const double per_col = (double)c->nb * (double)c->nnz * sizeof(float);
        cb = (int)std::min<double>(r, std::floor(budget / per_col));
        if (cb < r) cb &= ~7;   // budget-bound batches: whole 8-column partial rows
        if (cb < std::min(r, 32) || !psf_weights_fit(c->Mk, ((int64_t)cb + 31) / 32 * 32)) cb = 0;
    }
    if (cb == 0) {
        for (int i = 0; i < r; ++i) {
            fftt_status st = hess_apply(c, prec, isg2, static_cast<const char*>(X) + (size_t)i * N * es,
                                        dT, static_cast<char*>(Y) + (size_t)i * N * es);
            if (st != FFTT_OK) return st;
        }
        return FFTT_OK;
    }
    const int S = hess_slices(c->Mk, c->n_cu);
    ApplyArgs a = base_args(c);
    a.tab = staged_table_ptr(c, fmt);
    a.stage_q = (int)c->n_tx;
    for (int c0 = 0; c0 < r; c0 += cb) {
        const int n = std::min(cb, r - c0);
        const int64_t ldw = ((int64_t)n + 31) / 32 * 32;
        FFTT_HIP(c, c->d_hb_part.alloc((size_t)c->nb * c->nnz * hess_part_ld(n) * sizeof(float)));
        FFTT_HIP(c, c->d_hb_red.alloc((size_t)c->nb * S * c->Mk * n * sizeof(double)));
        FFTT_HIP(c, c->d_hb_w.alloc((size_t)c->nb * c->Mk * ldw * sizeof(float)));
        FFTT_HIP(c, launch_fill(c->stream, false, c->d_hb_w.p, (int64_t)c->nb * c->Mk * ldw));
        float* out = static_cast<float*>(Y) + (size_t)c0 * N;
        FFTT_HIP(c, launch_fill(c->stream, false, out, (int64_t)n * N));
        FFTT_HIP(c, launch_hess_block(c->stream, fmt, a, static_cast<const float*>(X) + (size_t)c0 * N,
                                      N, n, c->d_hb_part.as<float>(), c->d_gptr.as<int64_t>(),
                                      c->d_desc.p, S, c->d_hb_red.as<double>(),
                                      c->d_C.as<double>(), c->d_kptr.as<int32_t>(), isg2,
                                      c->d_hb_w.as<float>(), ldw, out));
    }
    return FFTT_OK;
}

// Orthonormal basis of the columns of Y ([l][N]) by the eigen-decomposition
// of the FP64 Gram matrix (G = U S U^T, Q = Y U_r S_r^-1/2 over the r
// eigenvalues above rel_tol S_max), done twice; the basis overwrites Y (the
// first pass goes through T).  Returns r.
fftt_status orth_block(fftt_ctx* c, bool fp64, void* Y, void* T, int l, double rel_tol,
                       int* r_out) {
    const int64_t N = c->Nm;
    int cols = l;
    for (int pass = 0; pass < 2; ++pass) {
        void* src = pass == 0 ? Y : T;
        void* dst = pass == 0 ? T : Y;
        FFTT_HIP(c, c->d_lr_part.alloc(gram_part_doubles(cols, cols, N) * sizeof(double)));
        FFTT_HIP(c, c->d_lr_small.alloc((size_t)cols * cols * sizeof(double)));
        FFTT_HIP(c, launch_gram(c->stream, fp64, src, cols, src, cols, N,
                                c->d_lr_part.as<double>(), c->d_lr_small.as<double>()));
        std::vector<double> G((size_t)cols * cols), w, U;
        FFTT_HIP(c, hipMemcpyAsync(G.data(), c->d_lr_small.p, G.size() * sizeof(double),
                                   hipMemcpyDeviceToHost, c->stream));
        FFTT_HIP(c, hipStreamSynchronize(c->stream));
        for (int a = 0; a < cols; ++a)   // exact symmetry before the eigensolver
            for (int b = a + 1; b < cols; ++b)
                G[(size_t)a * cols + b] = G[(size_t)b * cols + a] =
                    0.5 * (G[(size_t)a * cols + b] + G[(size_t)b * cols + a]);
        jacobi_eigh(G, cols, w, U);
        int r = 0;
        while (r < cols && w[r] > rel_tol * w[0] && w[r] > 0.0) ++r;
        if (r == 0) {
            *r_out = 0;
            return FFTT_OK;
        }
        std::vector<double> W((size_t)cols * r);
        for (int a = 0; a < cols; ++a)
            for (int b = 0; b < r; ++b) W[(size_t)a * r + b] = U[(size_t)a * cols + b] / std::sqrt(w[b]);
        FFTT_HIP(c, hipMemcpy(c->d_lr_small.p, W.data(), W.size() * sizeof(double),
                              hipMemcpyHostToDevice));
        FFTT_HIP(c, launch_combine(c->stream, fp64, src, cols, N, c->d_lr_small.as<double>(), r,
                                   dst));
        cols = r;
    }
    *r_out = cols;
    return FFTT_OK;
}

}  // namespace

// Solver iterations in a HIP graph: iteration 0 runs eagerly (it allocates
// the operators' work buffers); with `on`, iteration 1 is captured once on
// the context's stream and every later iteration replays the graph.  Event
// timing of the kernels is off while it lives.
struct IterGraph {
    fftt_ctx* c;
    bool on;
    bool prof;
    hipGraphExec_t exec = nullptr;
    ~IterGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        c->prof = prof;
    }
    template <class F>
    fftt_status step(int it, F&& body) {
        if (!on || it == 0) return body();
        if (!exec) {
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) {
                c->err = std::string("solve: graph capture: ") + hipGetErrorString(e);
                return FFTT_E_DEVICE;
            }
            const fftt_status sb = body();
            e = hipStreamEndCapture(c->stream, &g);
            if (sb != FFTT_OK) {
                if (g) (void)hipGraphDestroy(g);
                return sb;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                exec = nullptr;
                c->err = std::string("solve: graph: ") + hipGetErrorString(e);
                return FFTT_E_DEVICE;
            }
        }
        const hipError_t e = hipGraphLaunch(exec, c->stream);
        if (e != hipSuccess) {
            c->err = std::string("solve: graph launch: ") + hipGetErrorString(e);
            return FFTT_E_DEVICE;
        }
        return FFTT_OK;
    }
};

namespace {

// ---- work memory of fftt_apply_JT_noalloc ----
// A file-scope device array: every device the library runs on holds its own
// copy (kNoAllocScratch bytes) until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// for the symbol); it uses the device address that hipGetSymbolAddress
// returns for the current device, looked up once per device when the first
// context on it is created.
constexpr size_t kNoAllocScratch = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // by device ordinal; null until looked up

// Device address of this device's scratch array (device c->device current).
fftt_status init_scratch(fftt_ctx* c) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= c->device) g_scratch_ptr.resize(c->device + 1, nullptr);
    if (!g_scratch_ptr[c->device]) {
        void* p = nullptr;
        FFTT_HIP(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) FFTT_FAIL(c, FFTT_E_DEVICE, "scratch array has no device address");
        g_scratch_ptr[c->device] = p;
    }
    c->scratch = g_scratch_ptr[c->device];
    return FFTT_OK;
}

}  // namespace

extern "C" {

fftt_status fftt_create(fftt_ctx** out, int device, void* hip_stream) {
    if (!out) return FFTT_E_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return FFTT_E_DEVICE;
    fftt_ctx* c = new (std::nothrow) fftt_ctx();
    if (!c) return FFTT_E_NOMEM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return FFTT_E_DEVICE;
    }
    c->n_cu = prop.multiProcessorCount;
    c->lds_limit = prop.sharedMemPerBlock;
    if (set_device(c) != FFTT_OK || init_scratch(c) != FFTT_OK) {
        delete c;
        return FFTT_E_DEVICE;
    }
    *out = c;
    return FFTT_OK;
}

void fftt_destroy(fftt_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    delete c;
}

const char* fftt_last_error(const fftt_ctx* c) { return c ? c->err.c_str() : "null context"; }

fftt_status fftt_set_stream(fftt_ctx* c, void* hip_stream) {
    if (!c) return FFTT_E_INVALID;
    c->stream = static_cast<hipStream_t>(hip_stream);
    return FFTT_OK;
}

fftt_status fftt_set_geometry(fftt_ctx* c, double c0, const double* tx_xyz, int64_t n_tx,
                              const int32_t* pairs, int64_t n_pairs, const double origin[3],
                              const double spacing[3], const int64_t dims[3],
                              const uint8_t* active_mask) {
    if (!c) return FFTT_E_INVALID;
    if (!(c0 > 0) || !std::isfinite(c0)) FFTT_BAD(c, "c0 must be positive and finite");
    if (!tx_xyz || n_tx < 2 || n_tx > 65535) FFTT_BAD(c, "need 2 <= n_tx <= 65535 transducers");
    if (!pairs || n_pairs < 1 || n_pairs > INT32_MAX) FFTT_BAD(c, "need 1 <= n_pairs < 2^31");
    if (!origin || !spacing || !dims || !finite3(origin) || !finite3(spacing))
        FFTT_BAD(c, "grid origin/spacing must be finite");
    for (int k = 0; k < 3; ++k) {
        if (!(spacing[k] > 0)) FFTT_BAD(c, "grid spacing must be positive");
        if (dims[k] < 1 || dims[k] > (1 << 20)) FFTT_BAD(c, "grid dims out of range");
    }
    const int64_t N = dims[0] * dims[1] * dims[2];
    if (N > INT32_MAX) FFTT_BAD(c, "grid has more than 2^31 voxels");
    for (int64_t q = 0; q < n_tx; ++q)
        if (!finite3(tx_xyz + 3 * q)) FFTT_BAD(c, "non-finite transducer coordinate");
    for (int64_t i = 0; i < n_pairs; ++i) {
        const int32_t s = pairs[2 * i], r = pairs[2 * i + 1];
        if (s < 0 || r < 0 || s >= n_tx || r >= n_tx) FFTT_BAD(c, "pair index out of range");
        if (s == r) FFTT_BAD(c, "pair with source == receiver");
    }
    // no transducer may sit on an active voxel centre (the kernel is singular there)
    for (int64_t q = 0; q < n_tx; ++q) {
        int64_t idx[3];
        double d2 = 0.0;
        bool in = true;
        for (int k = 0; k < 3; ++k) {
            const double u = (tx_xyz[3 * q + k] - origin[k]) / spacing[k];
            idx[k] = (int64_t)std::llround(u);
            if (idx[k] < 0 || idx[k] >= dims[k]) in = false;
            const double d = (u - (double)idx[k]) * spacing[k];
            d2 += d * d;
        }
        if (in) {
            const int64_t v = idx[0] + dims[0] * (idx[1] + dims[1] * idx[2]);
            const bool act = active_mask ? active_mask[v] != 0 : true;
            const double hmin = std::min(spacing[0], std::min(spacing[1], spacing[2]));
            if (act && std::sqrt(d2) < 1e-3 * hmin)
                FFTT_BAD(c, "transducer " + std::to_string(q) + " lies on an active voxel centre");
        }
    }
    fftt_status st = set_device(c);
    if (st != FFTT_OK) return st;

    c->has_geom = false;
    c->lists_ok = false;
    c->c0 = c0;
    c->n_tx = n_tx;
    c->M = n_pairs;
    c->N = N;
    c->Nm = N;
    c->nxy2 = c->nz2 = 0;
    c->mask2.clear();
    c->tx.assign(tx_xyz, tx_xyz + 3 * n_tx);
    c->pairs_in.assign(pairs, pairs + 2 * n_pairs);
    c->dV = spacing[0] * spacing[1] * spacing[2];
    for (int k = 0; k < 3; ++k) {
        c->g.dims[k] = dims[k];
        c->g.origin[k] = origin[k];
        c->g.spacing[k] = spacing[k];
        c->g.ntile[k] = (dims[k] + kTile - 1) / kTile;
    }
    c->mask.assign((size_t)N, 1);
    if (active_mask) std::memcpy(c->mask.data(), active_mask, (size_t)N);
    std::vector<uint8_t> tact((size_t)(c->g.ntile[0] * c->g.ntile[1] * c->g.ntile[2]), 0);
    for (int64_t k = 0; k < dims[2]; ++k)
        for (int64_t j = 0; j < dims[1]; ++j)
            for (int64_t i = 0; i < dims[0]; ++i)
                if (c->mask[i + dims[0] * (j + dims[1] * k)])
                    tact[(i / kTile) + c->g.ntile[0] * ((j / kTile) + c->g.ntile[1] * (k / kTile))] = 1;
    c->act_tiles.clear();
    for (size_t t = 0; t < tact.size(); ++t)
        if (tact[t]) c->act_tiles.push_back((int32_t)t);
    // voxel index ranges covering every voxel outside the active tiles: the
    // batched PSFs zero these, then write all voxels of the active tiles, so
    // zeros written into active voxels are overwritten.  Each range is
    // widened to whole 128-byte lines, ranges closer than kFillGap voxels are
    // merged, and the result is split into pieces of at most kFillMax voxels
    // (one wavefront's share).
    constexpr int64_t kFillGap = 64, kFillMax = 4096;
    std::vector<int64_t> merged, runs;
    for (int64_t k = 0; k < dims[2]; ++k)
        for (int64_t j = 0; j < dims[1]; ++j) {
            const uint8_t* trow =
                tact.data() + c->g.ntile[0] * ((j / kTile) + c->g.ntile[1] * (k / kTile));
            const int64_t base = dims[0] * (j + dims[1] * k);
            for (int64_t i = 0; i < dims[0];) {
                if (trow[i / kTile]) { i = (i / kTile + 1) * kTile; continue; }
                int64_t e = i;
                while (e < dims[0] && !trow[e / kTile]) e = (e / kTile + 1) * kTile;
                e = std::min(e, dims[0]);
                // widened to whole 128-byte lines (32 floats)
                const int64_t rs = (base + i) & ~int64_t(31);
                const int64_t re = std::min(N, (base + e + 31) & ~int64_t(31));
                const size_t nr = merged.size();
                if (nr >= 2 && rs - (merged[nr - 2] + merged[nr - 1]) <= kFillGap) {
                    merged[nr - 1] = std::max(merged[nr - 1], re - merged[nr - 2]);
                } else {
                    merged.push_back(rs);
                    merged.push_back(re - rs);
                }
                i = e;
            }
        }
    for (size_t r = 0; r < merged.size(); r += 2)
        for (int64_t o = 0; o < merged[r + 1]; o += kFillMax) {
            runs.push_back(merged[r] + o);
            runs.push_back(std::min(kFillMax, merged[r + 1] - o));
        }
    c->n_fill_runs = (int64_t)runs.size() / 2;

    FFTT_HIP(c, c->d_tx.alloc(c->tx.size() * sizeof(double)));
    FFTT_HIP(c, c->d_mask.alloc((size_t)N));
    FFTT_HIP(c, c->d_tiles.alloc(std::max<size_t>(c->act_tiles.size(), 1) * sizeof(int32_t)));
    FFTT_HIP(c, hipMemcpy(c->d_tx.p, c->tx.data(), c->tx.size() * sizeof(double),
                          hipMemcpyHostToDevice));
    FFTT_HIP(c, hipMemcpy(c->d_mask.p, c->mask.data(), (size_t)N, hipMemcpyHostToDevice));
    if (!c->act_tiles.empty())
        FFTT_HIP(c, hipMemcpy(c->d_tiles.p, c->act_tiles.data(),
                              c->act_tiles.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    {
        // tile coordinates packed 21 bits each, read by the kernels instead
        // of dividing tile ids by the tile counts
        std::vector<uint64_t> ijk(std::max<size_t>(c->act_tiles.size(), 1), 0);
        const int64_t n0 = c->g.ntile[0], n1 = c->g.ntile[1];
        for (size_t k = 0; k < c->act_tiles.size(); ++k) {
            const int64_t t = c->act_tiles[k];
            ijk[k] = (uint64_t)(t % n0) | ((uint64_t)((t / n0) % n1) << 21) |
                     ((uint64_t)(t / (n0 * n1)) << 42);
        }
        FFTT_HIP(c, c->d_tile_ijk.alloc(ijk.size() * sizeof(uint64_t)));
        FFTT_HIP(c, hipMemcpy(c->d_tile_ijk.p, ijk.data(), ijk.size() * sizeof(uint64_t),
                              hipMemcpyHostToDevice));
    }
    FFTT_HIP(c, c->d_fill_runs.alloc(std::max<size_t>(runs.size(), 2) * sizeof(int64_t)));
    if (!runs.empty())
        FFTT_HIP(c, hipMemcpy(c->d_fill_runs.p, runs.data(), runs.size() * sizeof(int64_t),
                              hipMemcpyHostToDevice));
    st = build_pairs(c);
    if (st != FFTT_OK) return st;
    c->has_geom = true;
    return FFTT_OK;
}

fftt_status fftt_set_geometry_2d(fftt_ctx* c, double c0, const double* tx_xyz, int64_t n_tx,
                                 const int32_t* pairs, int64_t n_pairs, const double origin[2],
                                 const double spacing[2], const int64_t dims[2], double z0,
                                 double z1, int64_t nz, const uint8_t* active_mask) {
    if (!c) return FFTT_E_INVALID;
    if (!origin || !spacing || !dims) FFTT_BAD(c, "grid origin/spacing/dims missing");
    if (!std::isfinite(z0) || !std::isfinite(z1) || !(z1 > z0)) FFTT_BAD(c, "need z0 < z1");
    if (nz < 1 || nz > 4096) FFTT_BAD(c, "need 1 <= nz <= 4096 layers");
    if (dims[0] < 1 || dims[1] < 1 || dims[0] > (1 << 20) || dims[1] > (1 << 20))
        FFTT_BAD(c, "grid dims out of range");
    const int64_t nxy = dims[0] * dims[1];
    if (nxy * nz > INT32_MAX) FFTT_BAD(c, "prism has more than 2^31 voxels");
    // midpoint rule over [z0, z1]: layer k at z0 + (k + 1/2) dz
    const double dz = (z1 - z0) / (double)nz;
    const double o3[3] = {origin[0], origin[1], z0 + 0.5 * dz};
    const double s3[3] = {spacing[0], spacing[1], dz};
    const int64_t d3[3] = {dims[0], dims[1], nz};
    std::vector<uint8_t> m3;
    if (active_mask) {
        m3.resize((size_t)(nxy * nz));
        for (int64_t k = 0; k < nz; ++k) std::memcpy(m3.data() + k * nxy, active_mask, (size_t)nxy);
    }
    fftt_status st = fftt_set_geometry(c, c0, tx_xyz, n_tx, pairs, n_pairs, o3, s3, d3,
                                       active_mask ? m3.data() : nullptr);
    if (st != FFTT_OK) return st;
    c->Nm = c->nxy2 = nxy;
    c->nz2 = nz;
    c->mask2.assign((size_t)nxy, 1);
    if (active_mask) std::memcpy(c->mask2.data(), active_mask, (size_t)nxy);
    return FFTT_OK;
}

fftt_status fftt_set_kernel_table(fftt_ctx* c, int32_t band, const double* h, int64_t n,
                                  double r_max) {
    if (!c) return FFTT_E_INVALID;
    if (band < 0 || band >= kMaxBands) FFTT_BAD(c, "band out of range (0..3)");
    if (!h || n < 2 || n > kMaxTable) FFTT_BAD(c, "table length must be in 2..16384");
    if (!(r_max > 0) || !std::isfinite(r_max)) FFTT_BAD(c, "r_max must be positive and finite");
    for (int64_t k = 0; k < n; ++k)
        if (!std::isfinite(h[k])) FFTT_BAD(c, "non-finite table value");
    bool other = false;
    for (int b = 0; b < c->nb; ++b)
        if (b != band && c->band_set[b]) other = true;
    if (other && n != c->ntab) FFTT_BAD(c, "all bands must use the same table length");
    const double old_max = r_max_all(c);
    if (band >= c->nb) {
        c->nb = band + 1;
        c->h.resize(c->nb);
        c->r_max.resize(c->nb, 0.0);
        c->band_set.resize(c->nb, false);
        c->ser_a.resize(c->nb);
        c->ser_beta.resize(c->nb, 0.0);
    }
    if (c->r_max[band] != r_max) c->ser_a[band].clear();   // a series belongs to its r_max
    c->ntab = (int)n;
    c->h[band].assign(h, h + n);
    c->r_max[band] = r_max;
    c->band_set[band] = true;
    c->tab_dirty = true;
    if (r_max_all(c) != old_max) c->lists_ok = false;
    return FFTT_OK;
}

fftt_status fftt_build_table_from_pulse(double c0, const double* f, int64_t nt, double dt,
                                        int64_t n, double r_max, double* h_out,
                                        double* r_max_out) {
    std::string err;
    const int rc = build_table_from_pulse(c0, f, nt, dt, n, r_max, h_out, r_max_out, &err);
    return rc == 0 ? FFTT_OK : FFTT_E_INVALID;
}

fftt_status fftt_set_kernel_series(fftt_ctx* c, int32_t band, const double* a, int32_t n_terms,
                                   double beta, double r_max) {
    if (!c) return FFTT_E_INVALID;
    if (band < 0 || band >= c->nb || !c->band_set[band])
        FFTT_BAD(c, "set_kernel_series: the band's table must be set first");
    if (r_max != c->r_max[band]) FFTT_BAD(c, "set_kernel_series: r_max differs from the table's");
    if (!a || n_terms < 1 || n_terms > kSeriesMax) FFTT_BAD(c, "set_kernel_series: 1..64 terms");
    if (!(beta > 0) || !std::isfinite(beta) || beta * r_max > M_PI * (1.0 + 1e-12))
        FFTT_BAD(c, "set_kernel_series: need 0 < beta * r_max <= pi");
    for (int32_t m = 0; m < n_terms; ++m)
        if (!std::isfinite(a[m])) FFTT_BAD(c, "set_kernel_series: non-finite coefficient");
    c->ser_a[band].assign(a, a + n_terms);
    c->ser_beta[band] = beta;
    c->tab_dirty = true;
    return FFTT_OK;
}

fftt_status fftt_build_series_from_pulse(double c0, const double* f, int64_t nt, double dt,
                                         double r_max, double tol, int32_t max_terms,
                                         double* a_out, int32_t* n_terms_out, double* beta_out) {
    std::string err;
    const int rc = build_series_from_pulse(c0, f, nt, dt, r_max, tol, max_terms, a_out,
                                           n_terms_out, beta_out, &err);
    return rc == 0 ? FFTT_OK : FFTT_E_INVALID;
}

fftt_status fftt_coverage(fftt_ctx* c, fftt_precision prec, int32_t kind, void* out) {
    if (!c) return FFTT_E_INVALID;
    if (kind != 0 && kind != 1) FFTT_BAD(c, "coverage: kind must be 0 (sum |J|) or 1 (sum J^2)");
    if (!out) FFTT_BAD(c, "coverage: null output");
    if (prec != FFTT_FP32 && prec != FFTT_FP32_BF16TABLE) {
        if (prec == FFTT_FP64) FFTT_FAIL(c, FFTT_E_UNSUPPORTED, "coverage is computed in FP32");
        FFTT_BAD(c, "coverage: unknown precision");
    }
    fftt_status st = ensure_ready(c);
    if (st != FFTT_OK) return st;
    return coverage_one(c, prec, kind, static_cast<float*>(out));
}

fftt_status fftt_hessian_lowrank(fftt_ctx* c, fftt_precision prec, double noise_sigma,
                                 const void* omega, int32_t l, int32_t q, int32_t k,
                                 double* eigvals, void* eigvecs, int32_t* rank_out) {
    if (!c) return FFTT_E_INVALID;
    if (prec < FFTT_FP64 || prec > FFTT_FP32_BF16TABLE) FFTT_BAD(c, "lowrank: unknown precision");
    if (!omega || !eigvals || !eigvecs) FFTT_BAD(c, "lowrank: null argument");
    if (l < 1 || l > 512 || k < 1 || k > l || q < 0 || q > 32)
        FFTT_BAD(c, "lowrank: need 1 <= k <= l <= 512 and 0 <= q <= 32");
    if (!(noise_sigma > 0) || !std::isfinite(noise_sigma)) FFTT_BAD(c, "lowrank: noise_sigma must be > 0");
    fftt_status st = ensure_ready(c);
    if (st != FFTT_OK) return st;
    st = check_plane_precision(c, prec);
    if (st != FFTT_OK) return st;
    const bool fp64 = prec == FFTT_FP64;
    const size_t es = fp64 ? sizeof(double) : sizeof(float);
    const int64_t N = c->Nm, D = (int64_t)c->nb * c->M;
    const double isg2 = 1.0 / (noise_sigma * noise_sigma);
    // rank threshold on the Gram eigenvalues (squared singular values)
    const double tol = fp64 ? 1e-24 : 1e-12;
    FFTT_HIP(c, c->d_lr.alloc((size_t)2 * l * N * es));
    FFTT_HIP(c, c->d_solve.alloc((size_t)D * es));
    char* A = c->d_lr.as<char>();
    char* B = A + (size_t)l * N * es;
    void* dT = c->d_solve.p;
    // A = H Omega, orthonormalised
    st = hess_block(c, prec, isg2, omega, A, l, dT);
    if (st != FFTT_OK) return st;
    int r = 0;
    st = orth_block(c, fp64, A, B, l, tol, &r);
    if (st != FFTT_OK) return st;
    // subspace iterations: A = orth(H A)
    for (int it = 0; it < q && r > 0; ++it) {
        st = hess_block(c, prec, isg2, A, B, r, dT);
        if (st != FFTT_OK) return st;
        std::swap(A, B);
        st = orth_block(c, fp64, A, B, r, tol, &r);
        if (st != FFTT_OK) return st;
    }
    if (rank_out) *rank_out = r;
    std::vector<double> evals(k, 0.0);
    FFTT_HIP(c, launch_fill(c->stream, fp64, eigvecs, (int64_t)k * N));
    if (r > 0) {
        // Rayleigh-Ritz: T = Q^T H Q, T = U Theta U^T, Ritz vectors Q U
        st = hess_block(c, prec, isg2, A, B, r, dT);
        if (st != FFTT_OK) return st;
        FFTT_HIP(c, c->d_lr_part.alloc(gram_part_doubles(r, r, N) * sizeof(double)));
        FFTT_HIP(c, c->d_lr_small.alloc((size_t)r * r * sizeof(double)));
        FFTT_HIP(c, launch_gram(c->stream, fp64, A, r, B, r, N, c->d_lr_part.as<double>(),
                                c->d_lr_small.as<double>()));
        std::vector<double> T((size_t)r * r), w, U;
        FFTT_HIP(c, hipMemcpyAsync(T.data(), c->d_lr_small.p, T.size() * sizeof(double),
                                   hipMemcpyDeviceToHost, c->stream));
        FFTT_HIP(c, hipStreamSynchronize(c->stream));
        for (int a = 0; a < r; ++a)
            for (int b = a + 1; b < r; ++b)
                T[(size_t)a * r + b] = T[(size_t)b * r + a] =
                    0.5 * (T[(size_t)a * r + b] + T[(size_t)b * r + a]);
        jacobi_eigh(T, r, w, U);
        const int kk = std::min<int>(k, r);
        std::vector<double> Uk((size_t)r * kk);
        for (int a = 0; a < r; ++a)
            for (int b = 0; b < kk; ++b) Uk[(size_t)a * kk + b] = U[(size_t)a * r + b];
        for (int b = 0; b < kk; ++b) evals[b] = w[b];
        FFTT_HIP(c, hipMemcpy(c->d_lr_small.p, Uk.data(), Uk.size() * sizeof(double),
                              hipMemcpyHostToDevice));
        FFTT_HIP(c, launch_combine(c->stream, fp64, A, r, N, c->d_lr_small.as<double>(), kk,
                                   eigvecs));
    }
    FFTT_HIP(c, hipStreamSynchronize(c->stream));
    std::copy(evals.begin(), evals.end(), eigvals);
    return FFTT_OK;
}

fftt_status fftt_hessian_apply(fftt_ctx* c, fftt_precision prec, double noise_sigma,
                               const void* x, int32_t n_vec, void* y) {
    if (!c) return FFTT_E_INVALID;
    if (prec < FFTT_FP64 || prec > FFTT_FP32_BF16TABLE) FFTT_BAD(c, "hessian_apply: unknown precision");
    if (!x || !y || n_vec < 1) FFTT_BAD(c, "hessian_apply: null buffer or n_vec < 1");
    if (!(noise_sigma > 0) || !std::isfinite(noise_sigma))
        FFTT_BAD(c, "hessian_apply: noise_sigma must be > 0");
    fftt_status st = ensure_ready(c);
    if (st != FFTT_OK) return st;
    st = check_plane_precision(c, prec);
    if (st != FFTT_OK) return st;
    const size_t es = prec == FFTT_FP64 ? sizeof(double) : sizeof(float);
    FFTT_HIP(c, c->d_solve.alloc((size_t)c->nb * c->M * es));
    return hess_block(c, prec, 1.0 / (noise_sigma * noise_sigma), x, y, n_vec, c->d_solve.p);
}

fftt_status fftt_lowrank_diag(fftt_ctx* c, fftt_precision prec, const double* eigvals,
                              const void* eigvecs, int32_t k, double alpha, void* var_out,
                              void* res_out) {
    if (!c) return FFTT_E_INVALID;
    if (prec < FFTT_FP64 || prec > FFTT_FP32_BF16TABLE) FFTT_BAD(c, "lowrank_diag: unknown precision");
    if (!eigvals || !eigvecs || k < 1 || (!var_out && !res_out))
        FFTT_BAD(c, "lowrank_diag: null argument or k < 1");
    if (!(alpha > 0) || !std::isfinite(alpha)) FFTT_BAD(c, "lowrank_diag: alpha must be > 0");
    if (!c->has_geom) FFTT_FAIL(c, FFTT_E_STATE, "lowrank_diag: geometry not set");
    for (int32_t i = 0; i < k; ++i)
        if (!(eigvals[i] >= 0) || !std::isfinite(eigvals[i]))
            FFTT_BAD(c, "lowrank_diag: eigenvalues must be finite and >= 0");
    fftt_status st = set_device(c);
    if (st != FFTT_OK) return st;
    std::vector<double> d(k);
    for (int32_t i = 0; i < k; ++i) d[i] = eigvals[i] / (eigvals[i] + alpha);
    DevBuf dd;
    FFTT_HIP(c, dd.alloc((size_t)k * sizeof(double)));
    FFTT_HIP(c, hipMemcpy(dd.p, d.data(), d.size() * sizeof(double), hipMemcpyHostToDevice));
    FFTT_HIP(c, launch_lowrank_diag(c->stream, prec == FFTT_FP64, eigvecs, k, c->Nm,
                                    dd.as<double>(), 1.0 / alpha, var_out, res_out));
    // dd is freed on return: the kernel must have read it
    FFTT_HIP(c, hipStreamSynchronize(c->stream));
    return FFTT_OK;
}

fftt_status fftt_prepare(fftt_ctx* c) {
    if (!c) return FFTT_E_INVALID;
    return ensure_ready(c);
}

fftt_status fftt_work_count(fftt_ctx* c, int64_t* pv, int64_t* pv_evaluated, int64_t* lanes) {
    if (!c) return FFTT_E_INVALID;
    fftt_status st = ensure_ready(c);
    if (st != FFTT_OK) return st;
    if (pv) *pv = c->pv;
    if (pv_evaluated) *pv_evaluated = c->pv_eval;
    if (lanes) *lanes = c->lanes;
    return FFTT_OK;
}

fftt_status fftt_apply_J(fftt_ctx* c, fftt_precision prec, const void* dc, void* dT,
                         int32_t n_rhs) {
    if (!c) return FFTT_E_INVALID;
    if (prec < FFTT_FP64 || prec > FFTT_FP32_BF16TABLE) FFTT_BAD(c, "unknown precision");
    if (!dc || !dT || n_rhs < 1) FFTT_BAD(c, "apply_J: null buffer or n_rhs < 1");
    fftt_status st = ensure_ready(c);
    if (st != FFTT_OK) return st;
    st = check_plane_precision(c, prec);
    if (st != FFTT_OK) return st;
    if (const int cb = rhs_batch_cols(c, prec, false, n_rhs))
        return apply_rhs_batched(c, prec, false, dc, dT, n_rhs, cb);
    const size_t es = prec == FFTT_FP64 ? sizeof(double) : sizeof(float);
    for (int32_t r = 0; r < n_rhs; ++r) {
        st = apply_J_one(c, prec, static_cast<const char*>(dc) + (size_t)r * c->Nm * es,
                         static_cast<char*>(dT) + (size_t)r * c->nb * c->M * es);
        if (st != FFTT_OK) return st;
    }
    return FFTT_OK;
}

fftt_status fftt_apply_JT(fftt_ctx* c, fftt_precision prec, const void* dT, void* dc,
                          int32_t n_rhs) {
    if (!c) return FFTT_E_INVALID;
    if (prec < FFTT_FP64 || prec > FFTT_FP32_BF16TABLE) FFTT_BAD(c, "unknown precision");
    if (!dc || !dT || n_rhs < 1) FFTT_BAD(c, "apply_JT: null buffer or n_rhs < 1");
    fftt_status st = ensure_ready(c);
    if (st != FFTT_OK) return st;
    st = check_plane_precision(c, prec);
    if (st != FFTT_OK) return st;
    if (const int cb = rhs_batch_cols(c, prec, true, n_rhs))
        return apply_rhs_batched(c, prec, true, dT, dc, n_rhs, cb);
    const size_t es = prec == FFTT_FP64 ? sizeof(double) : sizeof(float);
    for (int32_t r = 0; r < n_rhs; ++r) {
        st = apply_JT_one(c, prec, static_cast<const char*>(dT) + (size_t)r * c->nb * c->M * es,
                          static_cast<char*>(dc) + (size_t)r * c->Nm * es);
        if (st != FFTT_OK) return st;
    }
    return FFTT_OK;
}

fftt_status fftt_apply_JT_noalloc(fftt_ctx* c, fftt_precision prec, const void* dT, void* dc,
                                  int32_t n_rhs) {
    if (!c) return FFTT_E_INVALID;
    if (prec < FFTT_FP64 || prec > FFTT_FP32_BF16TABLE) FFTT_BAD(c, "unknown precision");
    if (!dc || !dT || n_rhs < 1) FFTT_BAD(c, "apply_JT_noalloc: null buffer or n_rhs < 1");
    // everything ensure_ready would build must exist already
    if (!c->has_geom || c->nb == 0 || c->tab_dirty || !c->lists_ok)
        FFTT_FAIL(c, FFTT_E_STATE,
                  "apply_JT_noalloc: geometry and tables must be set and prepared "
                  "(fftt_prepare or an earlier apply)");
    for (int b = 0; b < c->nb; ++b)
        if (!c->band_set[b]) FFTT_FAIL(c, FFTT_E_STATE, "apply_JT_noalloc: a band has no table");
    fftt_status st = check_plane_precision(c, prec);
    if (st != FFTT_OK) return st;
    const size_t es = prec == FFTT_FP64 ? sizeof(double) : sizeof(float);
    const size_t wbytes = ((size_t)c->nb * c->Mk * es + 255) & ~(size_t)255;
    const size_t need = wbytes + (c->nxy2 ? (size_t)c->N * es : 0);
    if (need > kNoAllocScratch)
        FFTT_BAD(c, "apply_JT_noalloc: needs " + std::to_string(need) +
                        " bytes of work memory, more than the " +
                        std::to_string(kNoAllocScratch) + "-byte scratch array");
    if (!c->scratch) FFTT_FAIL(c, FFTT_E_STATE, "apply_JT_noalloc: no scratch address");
    st = set_device(c);
    if (st != FFTT_OK) return st;
    char* w = static_cast<char*>(c->scratch);
    for (int32_t r = 0; r < n_rhs; ++r) {
        st = apply_JT_work(c, prec, static_cast<const char*>(dT) + (size_t)r * c->nb * c->M * es,
                           static_cast<char*>(dc) + (size_t)r * c->Nm * es, w,
                           c->nxy2 ? w + wbytes : nullptr, false);
        if (st != FFTT_OK) return st;
    }
    return FFTT_OK;
}

fftt_status fftt_get_tuning(fftt_ctx* c, int32_t key, int32_t* value) {
    if (!c || !value) return FFTT_E_INVALID;
    switch (key) {
        case FFTT_TUNE_WAVES_PER_BLOCK: *value = c->waves_per_block; return FFTT_OK;
        case FFTT_TUNE_UNROLL_JT: *value = c->unroll_jt; return FFTT_OK;
        case FFTT_TUNE_UNROLL_J: *value = c->unroll_j; return FFTT_OK;
        case FFTT_TUNE_SPLIT_JT: *value = c->split_jt; return FFTT_OK;
        case FFTT_TUNE_SPLIT_J: *value = c->split_j; return FFTT_OK;
        case FFTT_TUNE_STAGED: *value = c->staged; return FFTT_OK;
        case FFTT_TUNE_UNROLL_JT_STAGED: *value = c->unroll_jts; return FFTT_OK;
        case FFTT_TUNE_UNROLL_J_STAGED: *value = c->unroll_js; return FFTT_OK;
        case FFTT_TUNE_STAGED_TABLE: *value = c->staged_pair_table; return FFTT_OK;
        case FFTT_TUNE_RECIPROCITY: *value = c->reciprocity; return FFTT_OK;
        case FFTT_TUNE_STAGED_BLOCK: *value = c->staged_block_max; return FFTT_OK;
        case FFTT_TUNE_KERNEL_EVAL: *value = c->eval_series; return FFTT_OK;
        case FFTT_TUNE_PSF_MATH: *value = c->psf_fp32_math; return FFTT_OK;
        case FFTT_TUNE_HESS_BATCHED: *value = c->hess_batched; return FFTT_OK;
        case FFTT_TUNE_RHS_BATCHED: *value = c->rhs_batched; return FFTT_OK;
        case FFTT_TUNE_ENTRY_ORDER: *value = c->entry_order; return FFTT_OK;
    }
    FFTT_BAD(c, "unknown tuning key");
}

// Mean time (ms) of `reps` launches of one operator's main kernel, after one
// untimed launch, under the current launch shape.
static fftt_status time_operator(fftt_ctx* c, fftt_precision prec, bool transpose, const void* x,
                                 void* y, int reps, double* ms) {
    fftt_status st = transpose ? apply_JT_one(c, prec, y, const_cast<void*>(x))
                               : apply_J_one(c, prec, x, y);
    if (st != FFTT_OK) return st;
    hipEvent_t e0, e1;
    FFTT_HIP(c, hipEventCreate(&e0));
    FFTT_HIP(c, hipEventCreate(&e1));
    FFTT_HIP(c, hipEventRecord(e0, c->stream));
    for (int r = 0; r < reps && st == FFTT_OK; ++r)
        st = transpose ? apply_JT_one(c, prec, y, const_cast<void*>(x)) : apply_J_one(c, prec, x, y);
    FFTT_HIP(c, hipEventRecord(e1, c->stream));
    FFTT_HIP(c, hipEventSynchronize(e1));
    float t = 0.f;
    FFTT_HIP(c, hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = t / reps;
    return st;
}

fftt_status fftt_autotune(fftt_ctx* c, fftt_precision prec, double max_seconds) {
    if (!c) return FFTT_E_INVALID;
    if (prec < FFTT_FP64 || prec > FFTT_FP32_BF16TABLE) FFTT_BAD(c, "autotune: unknown precision");
    if (!(max_seconds > 0)) FFTT_BAD(c, "autotune: max_seconds must be > 0");
    fftt_status st = ensure_ready(c);
    if (st != FFTT_OK) return st;
    st = check_plane_precision(c, prec);
    if (st != FFTT_OK) return st;
    const bool fp64 = prec == FFTT_FP64;
    const size_t es = fp64 ? sizeof(double) : sizeof(float);
    DevBuf xb, yb;
    FFTT_HIP(c, xb.alloc((size_t)c->Nm * es));
    FFTT_HIP(c, yb.alloc((size_t)c->nb * c->M * es));
    FFTT_HIP(c, launch_fill_value(c->stream, fp64, xb.p, c->Nm, 1.0));
    FFTT_HIP(c, launch_fill_value(c->stream, fp64, yb.p, (int64_t)c->nb * c->M, 1e-7));
    const bool prof = c->prof;
    c->prof = false;
    // the current shape is the baseline; its cost sets the repetitions
    double tj = 0, tjt = 0;
    st = time_operator(c, prec, false, xb.p, yb.p, 1, &tj);
    if (st == FFTT_OK) st = time_operator(c, prec, true, xb.p, yb.p, 1, &tjt);
    if (st != FFTT_OK) {
        c->prof = prof;
        return st;
    }
    const double per = std::max(tj + tjt, 1e-3);
    const int reps = std::max(1, std::min(5, (int)(0.05 * 1e3 * max_seconds / per)));
    auto t_start = std::chrono::steady_clock::now();
    auto budget_left = [&]() {
        const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start)
                              .count();
        return el < max_seconds;
    };
    struct Shape { int wpb, staged, table, uj, ujt, sj, sjt; };
    Shape best{c->waves_per_block, c->staged, c->staged_pair_table, 0, 0, c->split_j, c->split_jt};
    best.uj = c->staged ? c->unroll_js : c->unroll_j;
    best.ujt = c->staged ? c->unroll_jts : c->unroll_jt;
    double best_j = 1e30, best_jt = 1e30;
    const int wpbs[] = {16, 8, 4};
    const bool series = op_table(c, prec) == STAB_SERIES;   // needs the staged kernels
    const int tables = fp64 || series || prec == FFTT_FP32_BF16TABLE ? 1 : 2;
    for (int staged = 1; staged >= 0 && st == FFTT_OK; --staged) {
        if ((fp64 && staged) || (series && !staged)) continue;
        for (int wpb : wpbs) {
            for (int table = 0; table < (staged ? tables : 1); ++table) {
                c->waves_per_block = wpb;
                c->staged = staged;
                c->staged_pair_table = table;
                if (staged && !staged_q(c, prec)) continue;
                const int* us;
                static const int us_staged[] = {2, 4, 8, 0};
                static const int us_wave[] = {2, 4, 0};
                us = staged ? us_staged : us_wave;
                double bj = 1e30, bjt = 1e30;
                int buj = us[0], bujt = us[0], bsj = c->split_j, bsjt = c->split_jt;
                for (const int* u = us; *u && st == FFTT_OK && budget_left(); ++u) {
                    for (int split = staged ? 1 : 0; split <= 1; ++split) {
                        if (staged) {
                            c->unroll_js = c->unroll_jts = *u;
                        } else {
                            c->unroll_j = c->unroll_jt = *u;
                            c->split_j = c->split_jt = split;
                        }
                        double a = 0, b = 0;
                        st = time_operator(c, prec, false, xb.p, yb.p, reps, &a);
                        if (st == FFTT_OK) st = time_operator(c, prec, true, xb.p, yb.p, reps, &b);
                        if (st != FFTT_OK) break;
                        if (a < bj) { bj = a; buj = *u; bsj = split; }
                        if (b < bjt) { bjt = b; bujt = *u; bsjt = split; }
                    }
                }
                if (st == FFTT_OK && bj + bjt < best_j + best_jt) {
                    best_j = bj;
                    best_jt = bjt;
                    best = Shape{wpb, staged, table, buj, bujt, bsj, bsjt};
                }
            }
        }
    }
    c->prof = prof;
    c->waves_per_block = best.wpb;
    c->staged = best.staged;
    c->staged_pair_table = best.table;
    c->split_j = best.sj;
    c->split_jt = best.sjt;
    if (best.staged) {
        c->unroll_js = best.uj;
        c->unroll_jts = best.ujt;
    } else {
        c->unroll_j = best.uj;
        c->unroll_jt = best.ujt;
    }
    return st;
}

fftt_status fftt_set_tuning(fftt_ctx* c, int32_t key, int32_t value) {
    if (!c) return FFTT_E_INVALID;
    switch (key) {
        case FFTT_TUNE_WAVES_PER_BLOCK:
            if (value != 1 && value != 2 && value != 4 && value != 8 && value != 16)
                FFTT_BAD(c, "waves per block must be 1, 2, 4, 8 or 16");
            c->waves_per_block = value;
            return FFTT_OK;
        case FFTT_TUNE_UNROLL_JT:
        case FFTT_TUNE_UNROLL_J:
            if (value != 1 && value != 2 && value != 4) FFTT_BAD(c, "unroll must be 1, 2 or 4");
            (key == FFTT_TUNE_UNROLL_J ? c->unroll_j : c->unroll_jt) = value;
            return FFTT_OK;
        case FFTT_TUNE_STAGED:
            if (value != 0 && value != 1) FFTT_BAD(c, "staged must be 0 or 1");
            c->staged = value;
            return FFTT_OK;
        case FFTT_TUNE_UNROLL_JT_STAGED:
        case FFTT_TUNE_UNROLL_J_STAGED:
            if (value != 1 && value != 2 && value != 4 && value != 8)
                FFTT_BAD(c, "staged unroll must be 1, 2, 4 or 8");
            (key == FFTT_TUNE_UNROLL_J_STAGED ? c->unroll_js : c->unroll_jts) = value;
            return FFTT_OK;
        case FFTT_TUNE_STAGED_BLOCK:
            if (value != 0 && (value < 16 || (value & (value - 1)) != 0))
                FFTT_BAD(c, "staged block must be 0 or a power of two >= 16");
            c->staged_block_max = value;
            return FFTT_OK;
        case FFTT_TUNE_RECIPROCITY:
            if (value != 0 && value != 1) FFTT_BAD(c, "reciprocity must be 0 or 1");
            if (value != c->reciprocity) {
                c->reciprocity = value;
                if (c->has_geom) {
                    fftt_status st = set_device(c);
                    if (st != FFTT_OK) return st;
                    st = build_pairs(c);
                    if (st != FFTT_OK) return st;
                }
            }
            return FFTT_OK;
        case FFTT_TUNE_STAGED_TABLE:
            if (value != 0 && value != 1) FFTT_BAD(c, "staged table must be 0 or 1");
            c->staged_pair_table = value;
            return FFTT_OK;
        case FFTT_TUNE_KERNEL_EVAL:
            if (value != 0 && value != 1) FFTT_BAD(c, "kernel evaluation must be 0 or 1");
            c->eval_series = value;
            return FFTT_OK;
        case FFTT_TUNE_PSF_MATH:
            if (value != 0 && value != 1) FFTT_BAD(c, "PSF math must be 0 or 1");
            c->psf_fp32_math = value;
            return FFTT_OK;
        case FFTT_TUNE_HESS_BATCHED:
            if (value != 0 && value != 1) FFTT_BAD(c, "batched Hessian must be 0 or 1");
            c->hess_batched = value;
            return FFTT_OK;
        case FFTT_TUNE_RHS_BATCHED:
            if (value != 0 && value != 1) FFTT_BAD(c, "batched right-hand sides must be 0 or 1");
            c->rhs_batched = value;
            return FFTT_OK;
        case FFTT_TUNE_ENTRY_ORDER:
            if (value != 0 && value != 1) FFTT_BAD(c, "entry order must be 0 or 1");
            // the J^T copy is built with the lists: a change rebuilds them
            if (value != c->entry_order) c->lists_ok = false;
            c->entry_order = value;
            return FFTT_OK;
        case FFTT_TUNE_SPLIT_JT:
        case FFTT_TUNE_SPLIT_J:
            if (value != 0 && value != 1) FFTT_BAD(c, "split must be 0 or 1");
            (key == FFTT_TUNE_SPLIT_J ? c->split_j : c->split_jt) = value;
            return FFTT_OK;
    }
    FFTT_BAD(c, "unknown tuning key");
}

fftt_status fftt_profile(fftt_ctx* c, int32_t enable) {
    if (!c) return FFTT_E_INVALID;
    c->prof = enable != 0;
    for (auto& u : c->prof_used) u = 0;
    return FFTT_OK;
}

fftt_status fftt_kernel_time(fftt_ctx* c, int32_t which, double* ms, int64_t* launches) {
    if (!c) return FFTT_E_INVALID;
    if (which < 0 || which > 3 || !ms || !launches) FFTT_BAD(c, "kernel_time: bad argument");
    FFTT_HIP(c, hipStreamSynchronize(c->stream));
    double tot = 0.0;
    for (size_t i = 0; i < c->prof_used[which]; ++i) {
        float t = 0.f;
        FFTT_HIP(c, hipEventElapsedTime(&t, c->prof_ev[which][i].first,
                                        c->prof_ev[which][i].second));
        tot += t;
    }
    *ms = tot;
    *launches = (int64_t)c->prof_used[which];
    return FFTT_OK;
}

static fftt_status solve_impl(fftt_ctx* c, const fftt_solve_opts* o, const void* d_obs, void* x,
                              fftt_solve_report* rep);

fftt_status fftt_solve(fftt_ctx* c, const fftt_solve_opts* o, const void* d_obs, void* x,
                       fftt_solve_report* rep) {
    if (!c) return FFTT_E_INVALID;
    if (!o || !o->use_graph || c->stream != nullptr) return solve_impl(c, o, d_obs, x, rep);
    // the null stream cannot be captured: run on the context's private
    // stream, ordered after the caller's earlier work and before its later
    fftt_status st = set_device(c);
    if (st != FFTT_OK) return st;
    if (!c->graph_stream)
        FFTT_HIP(c, hipStreamCreateWithFlags(&c->graph_stream, hipStreamNonBlocking));
    hipEvent_t ev;
    FFTT_HIP(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ev, nullptr);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->graph_stream, ev, 0);
    if (e != hipSuccess) {
        (void)hipEventDestroy(ev);
        FFTT_HIP(c, e);
    }
    c->stream = c->graph_stream;
    st = solve_impl(c, o, d_obs, x, rep);
    c->stream = nullptr;
    e = hipEventRecord(ev, c->graph_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(nullptr, ev, 0);
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) FFTT_HIP(c, e);
    return st;
}

static fftt_status solve_impl(fftt_ctx* c, const fftt_solve_opts* o, const void* d_obs, void* x,
                              fftt_solve_report* rep) {
    if (!o || !d_obs || !x) FFTT_BAD(c, "solve: null argument");
    if (o->method != 0 && o->method != 1) FFTT_BAD(c, "solve: method must be 0 (CGLS) or 1 (LSQR)");
    if (o->prec < FFTT_FP64 || o->prec > FFTT_FP32_BF16TABLE) FFTT_BAD(c, "solve: unknown precision");
    if (!(o->noise_sigma > 0) || !std::isfinite(o->noise_sigma)) FFTT_BAD(c, "solve: noise_sigma must be > 0");
    if (!(o->alpha >= 0) || !std::isfinite(o->alpha)) FFTT_BAD(c, "solve: alpha must be >= 0");
    if (o->max_iter < 0) FFTT_BAD(c, "solve: max_iter < 0");
    if (o->precond != 0 && o->precond != 1) FFTT_BAD(c, "solve: precond must be 0 or 1");
    if (o->precond && o->method != 0) FFTT_BAD(c, "solve: the Jacobi preconditioner is for CGLS");
    fftt_status st = ensure_ready(c);
    if (st != FFTT_OK) return st;
    st = check_plane_precision(c, (fftt_precision)o->prec);
    if (st != FFTT_OK) return st;
    const fftt_precision prec = (fftt_precision)o->prec;
    const bool fp64 = prec == FFTT_FP64;
    const size_t es = fp64 ? sizeof(double) : sizeof(float);
    const int64_t N = c->Nm, D = (int64_t)c->nb * c->M;
    const double isg = 1.0 / o->noise_sigma, alpha = o->alpha;
    hipStream_t s = c->stream;
    // vectors: data-space r (or u), q; model-space sv, p (or v), w (or the
    // preconditioned residual z), minv
    FFTT_HIP(c, c->d_solve.alloc((size_t)(2 * D + 4 * N) * es));
    char* base = c->d_solve.as<char>();
    void* r = base;
    void* q = base + D * es;
    void* sv = base + 2 * D * es;
    void* p = base + (2 * D + N) * es;
    void* wv = base + (2 * D + 2 * N) * es;
    void* minv = base + (2 * D + 3 * N) * es;
    const bool pc = o->precond == 1;
    if (pc) {
        // Jacobi: M^-1 = 1 / (diag(J^T J) / sigma^2 + alpha), diagonal in FP32
        FFTT_HIP(c, c->d_diag.alloc((size_t)N * sizeof(float)));
        const fftt_precision dprec = prec == FFTT_FP32_BF16TABLE ? prec : FFTT_FP32;
        st = coverage_one(c, dprec, 1, c->d_diag.as<float>());
        if (st != FFTT_OK) return st;
        FFTT_HIP(c, solver_jacobi(c->stream, fp64, minv, c->d_diag.as<float>(), N, isg * isg,
                                  alpha));
    }
    FFTT_HIP(c, c->d_scal.alloc((32 + 512) * sizeof(double)));
    double* sc = c->d_scal.as<double>();
    double* part = sc + 32;
    FFTT_HIP(c, hipMemsetAsync(sc, 0, 32 * sizeof(double), s));
    const bool check = o->target_misfit > 0 || o->rel_tol > 0;
    double hs[32];
    auto fetch = [&]() -> fftt_status {
        FFTT_HIP(c, hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, s));
        FFTT_HIP(c, hipStreamSynchronize(s));
        return FFTT_OK;
    };
#define SOLVE_OK(expr)                       \
    do {                                     \
        fftt_status st_ = (expr);            \
        if (st_ != FFTT_OK) return st_;      \
    } while (0)
    IterGraph graph{c, o->use_graph != 0, c->prof};
    if (graph.on) c->prof = false;
    const auto t0 = std::chrono::steady_clock::now();
    int it = 0;
    double misfit = 0.0, relres = 0.0;
    if (o->method == 0) {
        // CGLS on (J^T J / sigma^2 + alpha I) x = J^T d / sigma^2; with the
        // Jacobi preconditioner the search directions follow z = M^-1 s and
        // gamma = s.z (PCG in CGLS form); SS, SS0 = |s|^2 for rel_tol
        enum { GAMMA = 0, DQ = 1, DP = 2, STEP = 3, BETA = 4, MIS = 5, G0 = 6, GNEW = 7,
               SS = 21, SS0 = 22 };
        void* zv = wv;
        if (o->use_x0) {
            SOLVE_OK(apply_J_one(c, prec, x, q));
            FFTT_HIP(c, solver_lin2(s, fp64, r, d_obs, q, D, isg, -isg));
        } else {
            FFTT_HIP(c, launch_fill(s, fp64, x, N));
            FFTT_HIP(c, solver_lin2(s, fp64, r, d_obs, nullptr, D, isg, 0.0));
        }
        SOLVE_OK(apply_JT_one(c, prec, r, sv));
        FFTT_HIP(c, solver_axpby(s, fp64, sv, x, N, isg, -1, -alpha, -1, sc));
        if (pc) {
            FFTT_HIP(c, solver_mul(s, fp64, zv, minv, sv, N));
            FFTT_HIP(c, solver_lin2(s, fp64, p, zv, nullptr, N, 1.0, 0.0));
            FFTT_HIP(c, solver_dot(s, fp64, sv, zv, N, part, sc, GAMMA, 1.0));
        } else {
            FFTT_HIP(c, solver_lin2(s, fp64, p, sv, nullptr, N, 1.0, 0.0));
            FFTT_HIP(c, solver_dot(s, fp64, sv, sv, N, part, sc, GAMMA, 1.0));
        }
        FFTT_HIP(c, solver_dot(s, fp64, sv, sv, N, part, sc, SS, 1.0));
        FFTT_HIP(c, solver_dot(s, fp64, sv, sv, N, part, sc, SS0, 1.0));
        FFTT_HIP(c, solver_dot(s, fp64, r, r, D, part, sc, MIS, 1.0));
        auto iteration = [&]() -> fftt_status {
            SOLVE_OK(apply_J_one(c, prec, p, q));
            FFTT_HIP(c, solver_dot(s, fp64, q, q, D, part, sc, DQ, isg * isg));
            FFTT_HIP(c, solver_dot(s, fp64, p, p, N, part, sc, DP, 1.0));
            FFTT_HIP(c, solver_cgls_step(s, sc, alpha));
            FFTT_HIP(c, solver_axpby(s, fp64, x, p, N, 1.0, -1, 1.0, STEP, sc));
            FFTT_HIP(c, solver_axpby(s, fp64, r, q, D, 1.0, -1, -isg, STEP, sc));
            SOLVE_OK(apply_JT_one(c, prec, r, sv));
            FFTT_HIP(c, solver_axpby(s, fp64, sv, x, N, isg, -1, -alpha, -1, sc));
            if (pc) {
                FFTT_HIP(c, solver_mul(s, fp64, zv, minv, sv, N));
                FFTT_HIP(c, solver_dot(s, fp64, sv, zv, N, part, sc, GNEW, 1.0));
                FFTT_HIP(c, solver_dot(s, fp64, sv, sv, N, part, sc, SS, 1.0));
            } else {
                FFTT_HIP(c, solver_dot(s, fp64, sv, sv, N, part, sc, GNEW, 1.0));
            }
            FFTT_HIP(c, solver_cgls_beta(s, sc));
            FFTT_HIP(c, solver_axpby(s, fp64, p, pc ? zv : sv, N, 1.0, BETA, 1.0, -1, sc));
            FFTT_HIP(c, solver_dot(s, fp64, r, r, D, part, sc, MIS, 1.0));
            return FFTT_OK;
        };
        // |s|^2 of the current residual (gamma itself without preconditioner)
        const int ss = pc ? SS : GAMMA;
        for (it = 0; it < o->max_iter;) {
            SOLVE_OK(graph.step(it, iteration));
            ++it;
            if (check) {
                SOLVE_OK(fetch());
                misfit = hs[MIS];
                relres = hs[SS0] > 0 ? std::sqrt(hs[ss] / hs[SS0]) : 0.0;
                if (o->target_misfit > 0 && misfit <= o->target_misfit) break;
                if (o->rel_tol > 0 && relres <= o->rel_tol) break;
            }
        }
        SOLVE_OK(fetch());
        misfit = hs[MIS];
        relres = hs[SS0] > 0 ? std::sqrt(hs[ss] / hs[SS0]) : 0.0;
    } else {
        // LSQR (Paige & Saunders) on A = J / sigma, b = d / sigma, damp = sqrt(alpha)
        enum { BETA = 8, ALPHA = 9, PHIBAR = 11, PHI_RHO = 12, THETA_RHO = 13, XX = 14,
               INV_BETA = 15, INV_ALPHA = 16, RES2 = 19, BNORM = 20 };
        const double damp = std::sqrt(alpha);
        if (o->use_x0) FFTT_BAD(c, "solve: LSQR starts from x0 = 0 (use_x0 must be 0)");
        FFTT_HIP(c, launch_fill(s, fp64, x, N));
        FFTT_HIP(c, solver_lin2(s, fp64, r, d_obs, nullptr, D, isg, 0.0));           // u = b
        FFTT_HIP(c, solver_dot(s, fp64, r, r, D, part, sc, BETA, 1.0));
        FFTT_HIP(c, solver_dot(s, fp64, r, r, D, part, sc, BNORM, 1.0));
        FFTT_HIP(c, solver_lsqr_beta(s, sc));
        FFTT_HIP(c, solver_axpby(s, fp64, r, r, D, 0.0, -1, 1.0, INV_BETA, sc));      // u /= beta
        SOLVE_OK(apply_JT_one(c, prec, r, sv));
        FFTT_HIP(c, solver_lin2(s, fp64, p, sv, nullptr, N, isg, 0.0));             // v = A^T u
        FFTT_HIP(c, solver_dot(s, fp64, p, p, N, part, sc, ALPHA, 1.0));
        FFTT_HIP(c, solver_lsqr_alpha_rot(s, sc, damp, 1));
        FFTT_HIP(c, solver_axpby(s, fp64, p, p, N, 0.0, -1, 1.0, INV_ALPHA, sc));     // v /= alpha
        FFTT_HIP(c, solver_lin2(s, fp64, wv, p, nullptr, N, 1.0, 0.0));             // w = v
        auto iteration = [&]() -> fftt_status {
            SOLVE_OK(apply_J_one(c, prec, p, q));
            FFTT_HIP(c, solver_axpby(s, fp64, r, q, D, -1.0, ALPHA, isg, -1, sc));   // u = Av - a u
            FFTT_HIP(c, solver_dot(s, fp64, r, r, D, part, sc, BETA, 1.0));
            FFTT_HIP(c, solver_lsqr_beta(s, sc));
            FFTT_HIP(c, solver_axpby(s, fp64, r, r, D, 0.0, -1, 1.0, INV_BETA, sc));
            SOLVE_OK(apply_JT_one(c, prec, r, sv));
            FFTT_HIP(c, solver_axpby(s, fp64, p, sv, N, -1.0, BETA, isg, -1, sc));   // v = A^T u - b v
            FFTT_HIP(c, solver_dot(s, fp64, p, p, N, part, sc, ALPHA, 1.0));
            FFTT_HIP(c, solver_lsqr_alpha_rot(s, sc, damp, 0));
            FFTT_HIP(c, solver_axpby(s, fp64, p, p, N, 0.0, -1, 1.0, INV_ALPHA, sc));
            FFTT_HIP(c, solver_axpby(s, fp64, x, wv, N, 1.0, -1, 1.0, PHI_RHO, sc));  // x += phi/rho w
            FFTT_HIP(c, solver_axpby(s, fp64, wv, p, N, 1.0, THETA_RHO, 1.0, -1, sc)); // w = v - theta/rho w
            return FFTT_OK;
        };
        for (it = 0; it < o->max_iter;) {
            SOLVE_OK(graph.step(it, iteration));
            ++it;
            if (check) {
                FFTT_HIP(c, solver_dot(s, fp64, x, x, N, part, sc, XX, 1.0));
                SOLVE_OK(fetch());
                misfit = hs[PHIBAR] * hs[PHIBAR] + hs[RES2] - alpha * hs[XX];
                relres = hs[BNORM] > 0 ? std::fabs(hs[PHIBAR]) / std::sqrt(hs[BNORM]) : 0.0;
                if (o->target_misfit > 0 && misfit <= o->target_misfit) break;
                if (o->rel_tol > 0 && relres <= o->rel_tol) break;
            }
        }
        FFTT_HIP(c, solver_dot(s, fp64, x, x, N, part, sc, XX, 1.0));
        SOLVE_OK(fetch());
        misfit = hs[PHIBAR] * hs[PHIBAR] + hs[RES2] - alpha * hs[XX];
        relres = hs[BNORM] > 0 ? std::fabs(hs[PHIBAR]) / std::sqrt(hs[BNORM]) : 0.0;
    }
#undef SOLVE_OK
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep) {
        rep->iters = it;
        rep->misfit = misfit;
        rep->rel_resid = relres;
        rep->time_ms = ms;
    }
    if (o->target_misfit > 0 && !(misfit <= o->target_misfit)) return FFTT_NOT_CONVERGED;
    if (o->target_misfit <= 0 && o->rel_tol > 0 && !(relres <= o->rel_tol)) return FFTT_NOT_CONVERGED;
    return FFTT_OK;
}

fftt_status fftt_psf(fftt_ctx* c, fftt_precision prec, const int64_t* voxels, int32_t n,
                     double noise_sigma, void* out) {
    if (!c) return FFTT_E_INVALID;
    if (prec < FFTT_FP64 || prec > FFTT_FP32_BF16TABLE) FFTT_BAD(c, "psf: unknown precision");
    if (!voxels || !out || n < 1) FFTT_BAD(c, "psf: null argument or n < 1");
    if (!(noise_sigma > 0) || !std::isfinite(noise_sigma)) FFTT_BAD(c, "psf: noise_sigma must be > 0");
    fftt_status st = ensure_ready(c);
    if (st != FFTT_OK) return st;
    st = check_plane_precision(c, prec);
    if (st != FFTT_OK) return st;
    const std::vector<uint8_t>& mk = c->nxy2 ? c->mask2 : c->mask;
    for (int32_t k = 0; k < n; ++k)
        if (voxels[k] < 0 || voxels[k] >= c->Nm || !mk[voxels[k]])
            FFTT_BAD(c, "psf: voxel index out of range or not active");
    const bool fp64 = prec == FFTT_FP64;
    const double s2 = 1.0 / (noise_sigma * noise_sigma);
    if (!fp64 && c->staged && !c->nxy2 &&
        psf_lds_bytes(c->nb, c->ntab, staged_table(c, prec), c->n_tx, c->psf_fp32_math == 0) <=
            c->lds_limit)
        return psf_batched(c, prec, voxels, n, s2, static_cast<float*>(out));
    const size_t es = fp64 ? sizeof(double) : sizeof(float);
    const int64_t D = (int64_t)c->nb * c->M;
    FFTT_HIP(c, c->d_solve.alloc((size_t)(D + c->Nm) * es));
    void* dT = c->d_solve.p;
    void* e = c->d_solve.as<char>() + D * es;
    for (int32_t k = 0; k < n; ++k) {
        FFTT_HIP(c, solver_unit(c->stream, fp64, e, c->Nm, voxels[k]));
        st = apply_J_one(c, prec, e, dT);
        if (st != FFTT_OK) return st;
        FFTT_HIP(c, solver_lin2(c->stream, fp64, dT, dT, nullptr, D, s2, 0.0));
        st = apply_JT_one(c, prec, dT, static_cast<char*>(out) + (size_t)k * c->Nm * es);
        if (st != FFTT_OK) return st;
    }
    return FFTT_OK;
}

}  // extern "C"
