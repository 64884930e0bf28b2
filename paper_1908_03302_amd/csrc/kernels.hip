// HIP kernels for gfx950: geometry pre-pass and the matrix-free traveltime
// Jacobian J (eq. forward_compact) and its transpose.
//
// Layout of the work: the voxel grid is cut into 4x4x4 tiles, one tile per
// wavefront (lane = voxel).  For every tile the pre-pass keeps the list of
// source-receiver pairs whose truncated kernel (detour R < R_max) can reach
// it.  Both operators walk that list: J^T accumulates sum_i J_ij dT_i in a
// register per voxel (no atomics), J reduces sum_j J_ij dc_j across the
// wavefront and writes one partial per (tile, pair), which a second kernel
// sums per pair in a fixed order.  Every kernel value is evaluated on the fly
// (Sec. II-C): A(x) from the two distances, h(R) from a table in LDS.
#include "internal.h"

#include <algorithm>
#include <type_traits>

namespace fftt {

// ----------------------------------------------------------------- helpers

__device__ __forceinline__ void tile_xyz(int64_t t, const GridGeom& g, int64_t& tx, int64_t& ty,
                                         int64_t& tz) {
    tx = t % g.ntile[0];
    ty = (t / g.ntile[0]) % g.ntile[1];
    tz = t / (g.ntile[0] * g.ntile[1]);
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, false);
}

// Sum over the 64 lanes of a wavefront (row butterflies, then row
// broadcasts); fixed order, so deterministic.  Result is wave-uniform.
__device__ __forceinline__ float wave_sum(float v) {
    v += __int_as_float(dpp_i<0xb1>(__float_as_int(v)));        // quad_perm 1,0,3,2
    v += __int_as_float(dpp_i<0x4e>(__float_as_int(v)));        // quad_perm 2,3,0,1
    v += __int_as_float(dpp_i<0x141>(__float_as_int(v)));       // row_half_mirror
    v += __int_as_float(dpp_i<0x140>(__float_as_int(v)));       // row_mirror
    v += __int_as_float(dpp_i<0x142, 0xa>(__float_as_int(v)));  // row_bcast:15
    v += __int_as_float(dpp_i<0x143, 0xc>(__float_as_int(v)));  // row_bcast:31
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i<CTRL, ROW_MASK>((int)(b & 0xffffffffll));
    const int hi = dpp_i<CTRL, ROW_MASK>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_d<0xb1>(v);
    v += dpp_d<0x4e>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    v += dpp_d<0x142, 0xa>(v);
    v += dpp_d<0x143, 0xc>(v);
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Swap the two 32-lane halves / the odd and even 16-lane rows and add: with
// the same register as both operands, the two results of the gfx950
// permlane swaps hold the two halves, so their sum is the cross-half sum.
__device__ __forceinline__ float add_halves(float x) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x),
                                                    false, false);
    x = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x),
                                                    false, false);
    return __uint_as_float(q[0]) + __uint_as_float(q[1]);
}

__device__ __forceinline__ double add_halves(double x) {
    const long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)(b & 0xffffffffll), hi = (unsigned)(b >> 32);
    const auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    x = __longlong_as_double(((long long)rh[0] << 32) | rl[0]) +
        __longlong_as_double(((long long)rh[1] << 32) | rl[1]);
    const long long c = __double_as_longlong(x);
    const unsigned lo2 = (unsigned)(c & 0xffffffffll), hi2 = (unsigned)(c >> 32);
    const auto ql = __builtin_amdgcn_permlane16_swap(lo2, lo2, false, false);
    const auto qh = __builtin_amdgcn_permlane16_swap(hi2, hi2, false, false);
    return __longlong_as_double(((long long)qh[0] << 32) | ql[0]) +
           __longlong_as_double(((long long)qh[1] << 32) | ql[1]);
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f(double v) {
    return dpp_d<CTRL>(v);
}

// Eight wavefront sums at once by halving the set of registers with every
// exchange.  permlane32_swap of registers a, b followed by one add leaves
// a's two 32-lane halves summed in lanes 0-31 and b's in lanes 32-63;
// permlane16_swap does the same for pairs of 16-lane rows.  The two
// remaining registers (four rows of partial sums each) are merged into one
// by summing each row's two halves (rotation by 8) and moving one register
// into the upper half of every row (DPP bank mask).  Every group of 8 lanes then
// holds partial sums of one value; two quad permutations and the row
// half-mirror (all symmetric, so no lane direction matters) leave the
// group's total in each of its lanes.  18 VALU instructions for 8 sums, no
// lane selects.  Group g (lanes 8g .. 8g + 7) ends with the total of value
// sum8_value_of_lane(8g).  Fixed order: deterministic.
__device__ __forceinline__ float swap32_add(float a, float b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b),
                                                    false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float swap16_add(float a, float b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b),
                                                    false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

template <int CTRL, int BANK_MASK>
__device__ __forceinline__ float dpp_move(float old, float src) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src),
                                                      CTRL, 0xf, BANK_MASK, false));
}

// Full-mask DPP move (zero "old": the compiler folds it into the consumer's
// add as one v_add_f32_dpp).
template <int CTRL>
__device__ __forceinline__ float dpp_all(float src) {
    return dpp_move<CTRL, 0xf>(0.f, src);
}

__device__ __forceinline__ float sum8_groups(const float (&v)[8]) {
    // s[k]: value 2k in lanes 0-31, 2k + 1 in lanes 32-63
    const float s0 = swap32_add(v[0], v[1]), s1 = swap32_add(v[2], v[3]);
    const float s2 = swap32_add(v[4], v[5]), s3 = swap32_add(v[6], v[7]);
    // t[j], rows 0..3: values 4j, 4j + 2, 4j + 1, 4j + 3
    const float t0 = swap16_add(s0, s1), t1 = swap16_add(s2, s3);
    // row halves summed: lanes 0-7 of row r then hold t0's row r, lanes 8-15
    // (banks 2 and 3, copied in by an identity move) t1's
    const float x0 = t0 + dpp_all<0x128>(t0);       // row_ror:8
    const float y0 = t1 + dpp_all<0x128>(t1);
    float x = dpp_move<0xe4, 0xc>(x0, y0);          // quad_perm 0,1,2,3
    x += dpp_all<0xb1>(x);                          // quad_perm 1,0,3,2
    x += dpp_all<0x4e>(x);                          // quad_perm 2,3,0,1
    x += dpp_all<0x141>(x);                         // row_half_mirror
    return x;
}

// Value held by the lanes of group g (lanes 8g .. 8g + 7) after
// sum8_groups: the group's half of its row picks t0 or t1, the row picks
// the value within it.
__device__ __forceinline__ int sum8_value_of_lane(int lane) {
    const int row = lane >> 4, half = (lane >> 3) & 1;
    return 4 * half + ((row & 1) << 1) + (row >> 1);
}

// U simultaneous wavefront sums: afterwards lane l holds sum_lanes v[l % U]
// (U = 1, 2 or 4).  Lanes are first paired so each lane carries one of the
// U sums, then the 64 / U lanes of each class are combined (row rotations by
// 4 and 8 keep l % 4, the half/row swaps finish).  Fixed order: deterministic.
template <int U, class T>
__device__ __forceinline__ T multi_sum(const T (&v)[U], int lane) {
    T x;
    if constexpr (U == 1) {
        x = v[0];
        x += dpp_f<0xb1>(x);                  // quad_perm 1,0,3,2  (lane ^ 1)
        x += dpp_f<0x4e>(x);                  // quad_perm 2,3,0,1  (lane ^ 2)
    } else if constexpr (U == 2) {
        const bool odd = lane & 1;
        x = odd ? v[1] : v[0];
        const T y = odd ? v[0] : v[1];
        x += dpp_f<0xb1>(y);
        x += dpp_f<0x4e>(x);
    } else if constexpr (U == 4) {
        const bool odd = lane & 1, two = lane & 2;
        T a = odd ? v[1] : v[0];
        const T b = odd ? v[0] : v[1];
        a += dpp_f<0xb1>(b);
        T c = odd ? v[3] : v[2];
        const T d = odd ? v[2] : v[3];
        c += dpp_f<0xb1>(d);
        x = two ? c : a;
        const T y = two ? a : c;
        x += dpp_f<0x4e>(y);
    } else {
        static_assert(U != 8 || !std::is_same<T, double>::value, "multi_sum<8>: FP32 only");
        static_assert(U == 8, "multi_sum: U in {1, 2, 4, 8}");
        return sum8_groups(v);
    }
    x += dpp_f<0x124>(x);                     // row_ror:4
    x += dpp_f<0x128>(x);                     // row_ror:8
    return add_halves(x);
}

// ------------------------------------------------- per (tile, transducer)

__global__ void k_txc(const int32_t* __restrict__ tiles, int64_t n_act,
                      const double* __restrict__ tx, int64_t n_tx, GridGeom g,
                      TxConst* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_act * n_tx) return;
    const int64_t a = i / n_tx, q = i - a * n_tx;
    int64_t tix, tiy, tiz;
    tile_xyz(tiles[a], g, tix, tiy, tiz);
    const double cx = g.origin[0] + ((double)(kTile * tix) + 1.5) * g.spacing[0];
    const double cy = g.origin[1] + ((double)(kTile * tiy) + 1.5) * g.spacing[1];
    const double cz = g.origin[2] + ((double)(kTile * tiz) + 1.5) * g.spacing[2];
    const double dx = cx - tx[3 * q], dy = cy - tx[3 * q + 1], dz = cz - tx[3 * q + 2];
    const double D2 = dx * dx + dy * dy + dz * dz;
    const float Df = (float)sqrt(D2);
    const double Dfd = (double)Df;
    TxConst c;
    c.d2x = 2.0 * dx;
    c.d2y = 2.0 * dy;
    c.d2z = 2.0 * dz;
    c.cq = D2 - Dfd * Dfd;
    c.D0f = Df;
    c.Q0f = (float)(Dfd * Dfd);
    out[i] = c;
}

hipError_t launch_txc(hipStream_t s, const int32_t* tiles, int64_t n_act, const double* tx,
                      int64_t n_tx, const GridGeom& g, TxConst* out) {
    const int64_t n = n_act * n_tx;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_txc, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tiles, n_act,
                       tx, n_tx, g, out);
    return hipGetLastError();
}

// ----------------------------------------------------------------- culling
//
// R(x) = |x - x_s| + |x - x_r| - L is convex, so over the box that holds the
// tile's voxel centres (half-widths hw) it is bounded below by its tangent
// plane at the centre: R >= R(c) - sum_k |dR/dx_k(c)| hw_k.  A pair is kept
// when that bound is below the cut radius; the list is in pair order.

template <bool FILL>
__global__ __launch_bounds__(256) void k_cull(const int32_t* __restrict__ tiles, int64_t n_act,
                                              const TxConst* __restrict__ txc, int64_t n_tx,
                                              const int32_t* __restrict__ ps,
                                              const int32_t* __restrict__ pr,
                                              const double* __restrict__ L, int64_t M,
                                              double hwx, double hwy, double hwz, double r_cut,
                                              int64_t* __restrict__ counts,
                                              const int64_t* __restrict__ tptr,
                                              Entry* __restrict__ ents) {
    __shared__ int s_wsum[4];
    const int64_t a = blockIdx.x;
    const TxConst* row = txc + a * n_tx;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = FILL ? tptr[a] : 0;
    int64_t count = 0;
    for (int64_t p0 = 0; p0 < M; p0 += 256) {
        const int64_t p = p0 + threadIdx.x;
        bool pass = false;
        double R0 = 0.0;
        uint32_t sr = 0;
        if (p < M) {
            const int s = ps[p], r = pr[p];
            const TxConst A = row[s], B = row[r];
            R0 = (double)A.D0f + (double)B.D0f - L[p];
            const double ia = 0.5 / (double)A.D0f, ib = 0.5 / (double)B.D0f;
            const double gx = A.d2x * ia + B.d2x * ib;
            const double gy = A.d2y * ia + B.d2y * ib;
            const double gz = A.d2z * ia + B.d2z * ib;
            const double lb = R0 - (fabs(gx) * hwx + fabs(gy) * hwy + fabs(gz) * hwz);
            pass = lb < r_cut;
            sr = (uint32_t)s | ((uint32_t)r << 16);
        }
        const unsigned long long bal = __ballot(pass);
        const int my = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) s_wsum[wave] = __popcll(bal);
        __syncthreads();
        int off = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int c = s_wsum[w];
            off += (w < wave) ? c : 0;
            tot += c;
        }
        if (FILL && pass) {
            const float hi = (float)R0;
            const float lo = (float)(R0 - (double)hi);
            Entry E;
            E.p = (int32_t)p;
            E.sr = sr;
            E.R0hi = hi;
            E.R0lo = lo;
            ents[base + count + off + my] = E;
        }
        count += tot;
        __syncthreads();
    }
    if (!FILL && threadIdx.x == 0) counts[a] = count;
}

hipError_t launch_cull(hipStream_t s, bool fill, const int32_t* tiles, int64_t n_act,
                       const TxConst* txc, int64_t n_tx, const int32_t* ps, const int32_t* pr,
                       const double* L, int64_t M, const GridGeom& g, double r_cut,
                       int64_t* counts, const int64_t* tptr, Entry* ents) {
    if (n_act == 0) return hipSuccess;
    const double hwx = 0.5 * (kTile - 1) * g.spacing[0];
    const double hwy = 0.5 * (kTile - 1) * g.spacing[1];
    const double hwz = 0.5 * (kTile - 1) * g.spacing[2];
    if (fill)
        hipLaunchKernelGGL(k_cull<true>, dim3((unsigned)n_act), dim3(256), 0, s, tiles, n_act,
                           txc, n_tx, ps, pr, L, M, hwx, hwy, hwz, r_cut, counts, tptr, ents);
    else
        hipLaunchKernelGGL(k_cull<false>, dim3((unsigned)n_act), dim3(256), 0, s, tiles, n_act,
                           txc, n_tx, ps, pr, L, M, hwx, hwy, hwz, r_cut, counts, tptr, ents);
    return hipGetLastError();
}

// ------------------------------------------------ per-chunk count scan
//
// Deterministic compaction used by the reduction index: tiles are grouped in
// chunks, each chunk counts per key, counts are scanned across chunks per key
// (exclusive, in place) and the chunks later hand out slots tile by tile.

__global__ void k_chunk_scan(int32_t* __restrict__ cnt, int64_t n_chunks, int64_t K,
                             int64_t* __restrict__ total) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= K) return;
    int64_t run = 0;
    for (int64_t c = 0; c < n_chunks; ++c) {
        const int32_t v = cnt[c * K + p];
        cnt[c * K + p] = (int32_t)run;
        run += v;
    }
    total[p] = run;
}

hipError_t launch_chunk_scan(hipStream_t s, int32_t* cnt, int64_t n_chunks, int64_t K,
                             int64_t* total) {
    hipLaunchKernelGGL(k_chunk_scan, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, cnt,
                       n_chunks, K, total);
    return hipGetLastError();
}

// --------------------------------------------------------------- work count

// Voxel of `lane` in active tile a: the tile's coordinates come packed from
// the host (21 bits each), so no kernel divides by the tile counts.
__device__ __forceinline__ void voxel_of_lane(const ApplyArgs& A, int64_t a, int lane,
                                              bool& inside, bool& act, int64_t& vidx,
                                              int64_t v[3]) {
    const uint64_t ijk = A.tile_ijk[a];
    v[0] = kTile * (int64_t)(ijk & kTileCoordMask) + (lane & 3);
    v[1] = kTile * (int64_t)((ijk >> 21) & kTileCoordMask) + ((lane >> 2) & 3);
    v[2] = kTile * (int64_t)(ijk >> 42) + (lane >> 4);
    inside = v[0] < A.g.dims[0] && v[1] < A.g.dims[1] && v[2] < A.g.dims[2];
    vidx = inside ? v[0] + A.g.dims[0] * (v[1] + A.g.dims[1] * v[2]) : 0;
    act = inside && A.mask[vidx] != 0;
}

// pv_eval counts the (kernel pair, active voxel) evaluations with detour
// below rmax; pv_op the same over caller pairs (a kernel pair stands for
// kptr[p+1] - kptr[p] caller pairs with identical rows).
__global__ __launch_bounds__(256) void k_count_pv(ApplyArgs A, double rmax,
                                                  const double* __restrict__ L,
                                                  const int32_t* __restrict__ ps,
                                                  const int32_t* __restrict__ pr,
                                                  const double* __restrict__ tx,
                                                  const int32_t* __restrict__ kptr,
                                                  unsigned long long* pv_op,
                                                  unsigned long long* pv_eval) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t a = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (a >= A.n_act) return;
    bool inside, act;
    int64_t vidx, v[3];
    voxel_of_lane(A, a, lane, inside, act, vidx, v);
    const double x = A.g.origin[0] + (double)v[0] * A.g.spacing[0];
    const double y = A.g.origin[1] + (double)v[1] * A.g.spacing[1];
    const double z = A.g.origin[2] + (double)v[2] * A.g.spacing[2];
    unsigned long long cnt = 0, cop = 0;
    for (int64_t e = A.tptr[a]; e < A.tptr[a + 1]; ++e) {
        const int p = A.ents[e].p;
        const double* xs = tx + 3 * ps[p];
        const double* xr = tx + 3 * pr[p];
        const double Rs = sqrt((x - xs[0]) * (x - xs[0]) + (y - xs[1]) * (y - xs[1]) +
                               (z - xs[2]) * (z - xs[2]));
        const double Rr = sqrt((x - xr[0]) * (x - xr[0]) + (y - xr[1]) * (y - xr[1]) +
                               (z - xr[2]) * (z - xr[2]));
        const bool in = act && (Rs + Rr - L[p] < rmax);
        const unsigned long long k = __popcll(__ballot(in));
        cnt += k;
        cop += k * (unsigned long long)(kptr[p + 1] - kptr[p]);
    }
    if (lane == 0) {
        atomicAdd(pv_eval, cnt);
        atomicAdd(pv_op, cop);
    }
}

hipError_t launch_count_pv(hipStream_t s, const ApplyArgs& a, double r_max_all,
                           const double* L, const int32_t* ps, const int32_t* pr,
                           const double* tx, const int32_t* kptr, unsigned long long* pv_op,
                           unsigned long long* pv_eval) {
    if (a.n_act == 0) return hipSuccess;
    const unsigned nblk = (unsigned)((a.n_act + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL(k_count_pv, dim3(nblk), dim3(64 * kWavesPerBlock), 0, s, a, r_max_all, L,
                       ps, pr, tx, kptr, pv_op, pv_eval);
    return hipGetLastError();
}

// ------------------------------------------------------- small vector kernels

// J^T weights of the kernel pairs: w[b][k] = C_k sum of dT[b][i] over the
// caller pairs i of group k (pairs with identical rows, e.g. (s, r) and
// (r, s)), summed in FP64 in group order.
template <class T>
__global__ void k_weights(const T* __restrict__ dT, const int32_t* __restrict__ kptr,
                          const int32_t* __restrict__ kidx, const double* __restrict__ C,
                          int64_t Mk, int64_t M, int nb, T* __restrict__ w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Mk * nb) return;
    const int64_t b = i / Mk, k = i - b * Mk;
    double t = 0.0;
    for (int32_t j = kptr[k]; j < kptr[k + 1]; ++j) t += (double)dT[b * M + kidx[j]];
    w[i] = (T)(C[k] * t);
}

hipError_t launch_weights(hipStream_t s, bool fp64, const void* dT, const int32_t* kptr,
                          const int32_t* kidx, const double* C, int64_t Mk, int64_t M, int nb,
                          void* w) {
    const int64_t n = Mk * nb;
    const unsigned nblk = (unsigned)((n + 255) / 256);
    if (fp64)
        hipLaunchKernelGGL(k_weights<double>, dim3(nblk), dim3(256), 0, s, (const double*)dT,
                           kptr, kidx, C, Mk, M, nb, (double*)w);
    else
        hipLaunchKernelGGL(k_weights<float>, dim3(nblk), dim3(256), 0, s, (const float*)dT,
                           kptr, kidx, C, Mk, M, nb, (float*)w);
    return hipGetLastError();
}

template <class T>
__global__ void k_fill0(T* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (T)0;
}

template <class T>
__global__ void k_fillv(T* __restrict__ p, int64_t n, T v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_value(hipStream_t s, bool fp64, void* p, int64_t n, double v) {
    if (n == 0) return hipSuccess;
    const unsigned nblk = (unsigned)((n + 255) / 256);
    if (fp64)
        hipLaunchKernelGGL(k_fillv<double>, dim3(nblk), dim3(256), 0, s, (double*)p, n, v);
    else
        hipLaunchKernelGGL(k_fillv<float>, dim3(nblk), dim3(256), 0, s, (float*)p, n, (float)v);
    return hipGetLastError();
}

template <class T>
__global__ void k_sum_z(const T* __restrict__ in, int64_t nxy, int64_t nz, T* __restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nxy) return;
    double s = 0.0;
    for (int64_t k = 0; k < nz; ++k) s += (double)in[p + k * nxy];
    out[p] = (T)s;
}

hipError_t launch_sum_z(hipStream_t s, bool fp64, const void* in, int64_t nxy, int64_t nz,
                        void* out) {
    if (nxy == 0) return hipSuccess;
    const unsigned nblk = (unsigned)((nxy + 255) / 256);
    if (fp64)
        hipLaunchKernelGGL(k_sum_z<double>, dim3(nblk), dim3(256), 0, s, (const double*)in, nxy,
                           nz, (double*)out);
    else
        hipLaunchKernelGGL(k_sum_z<float>, dim3(nblk), dim3(256), 0, s, (const float*)in, nxy, nz,
                           (float*)out);
    return hipGetLastError();
}

hipError_t launch_fill(hipStream_t s, bool fp64, void* p, int64_t n) {
    if (n == 0) return hipSuccess;
    const unsigned nblk = (unsigned)((n + 255) / 256);
    if (fp64)
        hipLaunchKernelGGL(k_fill0<double>, dim3(nblk), dim3(256), 0, s, (double*)p, n);
    else
        hipLaunchKernelGGL(k_fill0<float>, dim3(nblk), dim3(256), 0, s, (float*)p, n);
    return hipGetLastError();
}

// ------------------------------------------------------ kernel evaluation

// FP32 path: the distance to a transducer is split as R_x = D0f + delta with
// delta = n / (R_x + D0f), n formed in FP64 from the tile-relative geometry,
// so the detour R = R0 + delta_s + delta_r never subtracts large numbers.
__device__ __forceinline__ void dist32(const TxConst& c, double ux, double uy, double uz,
                                       double uu, float& delta, float& rs) {
    const double n = fma(c.d2x, ux, fma(c.d2y, uy, fma(c.d2z, uz, uu + c.cq)));
    const float nf = (float)n;
    const float q = c.Q0f + nf;
    rs = __builtin_amdgcn_rsqf(q);
    const float Rx = q * rs;
    delta = nf * __builtin_amdgcn_rcpf(Rx + c.D0f);
}

// FP64 path: plain distances (FP64 leaves no cancellation that matters),
// returned as delta = R_x - D0f and 1/R_x.  R_x and 1/R_x come together from
// the hardware reciprocal square root estimate y (relative error below
// 2^-23) and two steps of Goldschmidt's coupled iteration on g ~ sqrt(s),
// h ~ 1/(2 sqrt(s)): r = 1/2 - g h, g += g r, h += h r.  Each step squares the
// relative error, so two reach the precision of a double to a few ulp; no
// division and no range scaling (s is a squared distance of order 1e-4 m^2,
// far from the limits of the format).
__device__ __forceinline__ void dist64(const TxConst& c, double ux, double uy, double uz,
                                       double uu, double& delta, double& inv_r) {
    const double n = fma(c.d2x, ux, fma(c.d2y, uy, fma(c.d2z, uz, uu + c.cq)));
    const double D = (double)c.D0f;
    const double s = fma(D, D, n);
    const double y = __builtin_amdgcn_rsq(s);
    double g = s * y, h = 0.5 * y;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double r = fma(-g, h, 0.5);
        g = fma(g, r, g);
        h = fma(h, r, h);
    }
    delta = g - D;
    inv_r = h + h;
}

// Table coordinate x = R / dR clamped to [0, n-1] (v_med3; a NaN maps into
// range).  The lookups below take the clamped coordinate; the interpolation
// weight is fract(x), exact for x >= 0.
__device__ __forceinline__ float table_x(float x, float nm1) {
    return __builtin_amdgcn_fmed3f(x, 0.0f, nm1);
}

// Linear interpolation in a table of nodes k = 0..n-1 over [0, r_max]; entry
// k stores (h_k, h_{k+1} - h_k) and entry n-1 is (0, 0), so clamping the
// coordinate to n-1 yields zero for every R >= r_max.
__device__ __forceinline__ float lookup_x(const float2* tab, float x, float) {
    const int k = (int)x;
    const float2 t = tab[k];
    return fmaf(__builtin_amdgcn_fractf(x), t.y, t.x);
}

// BF16 table: entry k packs a = bf16(h_k) in the low half and
// d = bf16(h_{k+1} - a) in the high half, so h = a + f d; the rounding of a
// is fully felt at the node and fades linearly to the next node.
__device__ __forceinline__ float lookup_x(const uint32_t* tab, float x, float) {
    const int k = (int)x;
    const uint32_t e = tab[k];
    return fmaf(__builtin_amdgcn_fractf(x), __uint_as_float(e & 0xffff0000u),
                __uint_as_float(e << 16));
}

// FP32 node table h_0..h_{n-1}, h_n = 0 (one float per node, half the LDS of
// the (h, slope) layout): both nodes come from one ds_read2; the truncation
// to zero for R >= r_max is a select on the interpolated value (the reads
// themselves are never predicated: k <= n-1 always).
__device__ __forceinline__ float lookup_x(const float* tab, float x, float nm1) {
    const int k = (int)x;
    const float h0 = tab[k], h1 = tab[k + 1];
    const float v = fmaf(__builtin_amdgcn_fractf(x), h1 - h0, h0);
    return x < nm1 ? v : 0.0f;
}

// FP32 node table whose top node h_{n-1} is stored as 0 (used when every
// band's h at r_max is negligible): a coordinate clamped to n-1 reads
// (0, next) with weight fract(x) = 0, so the truncation needs no select.
// The float after a band's top node must be finite: the next band's first
// node, the table's zeroed alignment padding, or the staged distances.
struct NodeZ {
    float v;
};

__device__ __forceinline__ float lookup_x(const NodeZ* tab, float x, float) {
    const int k = (int)x;
    const float h0 = tab[k].v, h1 = tab[k + 1].v;
    return fmaf(__builtin_amdgcn_fractf(x), h1 - h0, h0);
}

// Sine series instead of a table (the paper's own stored form of eq.
// Kernel_freq, Sec. II-C):  h = sum_{m=1}^{n} a_m sin(m theta), theta = beta R,
// h = 0 for R >= r_max.  Per band, kSeriesStride floats in global memory:
// [theta/2 per unit of the table coordinate, n (int bits, a multiple of 4),
// 0, 0, a_1 .. a_n].  They are read through the constant address space, so
// the wave-uniform coefficients arrive by scalar loads as SGPR operands.
// Clenshaw's recurrence in Reinsch's form: with
// lam = 2 cos(theta) - 2 = -4 sin^2(theta/2),
//   d_m = a_m + lam b_{m+1} + d_{m+1},  b_m = d_m + b_{m+1},  h = b_1 sin(theta),
// which, unlike the three-term form b_m = a_m + 2 cos(theta) b_{m+1} - b_{m+2},
// does not amplify rounding as theta -> 0 (3 VALU per term).  sin and cos of
// theta/2 <= pi/2 come from their Taylor polynomials to degree 13 / 14
// (truncation < 1e-9).
struct SinCoef {
    float v;
};

template <class TabT>
constexpr bool table_in_lds() { return true; }
template <>
constexpr bool table_in_lds<SinCoef>() { return false; }

typedef float f32x4v __attribute__((ext_vector_type(4)));
using ConstF = const __attribute__((address_space(4))) float;
using ConstF4 = const __attribute__((address_space(4))) f32x4v;

// Half-angle sine and cosine for 0 <= t <= pi/2 (Taylor polynomials).
__device__ __forceinline__ void half_angle(float t, float& sh, float& ch) {
    // 1/k! for the Taylor polynomials
    constexpr float f3 = 1.0 / 6, f5 = 1.0 / 120, f7 = 1.0 / 5040, f9 = 1.0 / 362880,
                    f11 = 1.0 / 39916800, f13 = 1.0 / 6227020800.0;
    constexpr float f2 = 1.0 / 2, f4 = 1.0 / 24, f6 = 1.0 / 720, f8 = 1.0 / 40320,
                    f10 = 1.0 / 3628800, f12 = 1.0 / 479001600, f14 = 1.0 / 87178291200.0;
    const float u = t * t;
    float sp = fmaf(u, -f13, f11);
    sp = fmaf(u, sp, -f9);
    sp = fmaf(u, sp, f7);
    sp = fmaf(u, sp, -f5);
    sp = fmaf(u, sp, f3);
    sp = fmaf(u, -sp, 1.0f);
    float cp = fmaf(u, f14, -f12);
    cp = fmaf(u, cp, f10);
    cp = fmaf(u, cp, -f8);
    cp = fmaf(u, cp, f6);
    cp = fmaf(u, cp, -f4);
    cp = fmaf(u, cp, f2);
    ch = fmaf(u, -cp, 1.0f);
    sh = t * sp;
}

// U lookups at once (table coordinates x[u], unclamped).  For the tables
// these are independent interpolations; the series evaluates the U
// recurrences together, so every scalar load of four coefficients serves
// all of them.
template <int U, class TabT>
__device__ __forceinline__ void lookup_n(const TabT* tab, const float (&x)[U], float nm1,
                                         float (&h)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) h[u] = lookup_x(tab, table_x(x[u], nm1), nm1);
}

template <int U>
__device__ __forceinline__ void lookup_n(const SinCoef* tab, const float (&x)[U], float nm1,
                                         float (&h)[U]) {
    ConstF* c = (ConstF*)tab;
    float xc[U], lam[U], sn[U], b[U], d[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        xc[u] = table_x(x[u], nm1);
        float sh, ch;
        half_angle(c[0] * xc[u], sh, ch);  // theta / 2
        lam[u] = -4.0f * sh * sh;
        sn[u] = 2.0f * sh * ch;            // sin(theta)
        b[u] = d[u] = 0.0f;
    }
    const int n = __float_as_int(c[1]);
    for (int k = n; k > 0; k -= 4) {
        const f32x4v a = *(ConstF4*)(c + k);   // a_{k-3} .. a_k
#pragma unroll
        for (int u = 0; u < U; ++u) {
            d[u] = fmaf(lam[u], b[u], a.w + d[u]);
            b[u] += d[u];
            d[u] = fmaf(lam[u], b[u], a.z + d[u]);
            b[u] += d[u];
            d[u] = fmaf(lam[u], b[u], a.y + d[u]);
            b[u] += d[u];
            d[u] = fmaf(lam[u], b[u], a.x + d[u]);
            b[u] += d[u];
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) h[u] = xc[u] < nm1 ? b[u] * sn[u] : 0.0f;
}

// Band b's table (or series) within a staged kernel's table pointer.
template <class TabT>
__device__ __forceinline__ const TabT* band_tab(const TabT* st, int b, int ntab) {
    return st + (size_t)b * (table_in_lds<TabT>() ? ntab : kSeriesStride);
}

template <class TabT>
__device__ __forceinline__ float lookup(const TabT* tab, float R, float inv_dr, float nm1) {
    return lookup_x(tab, table_x(R * inv_dr, nm1), nm1);
}

__device__ __forceinline__ double lookup(const double2* tab, double R, double inv_dr, double nm1) {
    const double x = fmin(fmax(R * inv_dr, 0.0), nm1);
    const int k = (int)x;
    const double f = x - (double)k;
    const double2 t = tab[k];
    return fma(f, t.y, t.x);
}

struct LaneVox {
    bool inside, act;
    int64_t vidx;
    double ux, uy, uz, uu;
};

__device__ __forceinline__ LaneVox lane_vox(const ApplyArgs& A, int64_t a, int lane) {
    LaneVox L;
    int64_t v[3];
    voxel_of_lane(A, a, lane, L.inside, L.act, L.vidx, v);
    L.ux = ((double)(lane & 3) - 1.5) * A.g.spacing[0];
    L.uy = ((double)((lane >> 2) & 3) - 1.5) * A.g.spacing[1];
    L.uz = ((double)(lane >> 4) - 1.5) * A.g.spacing[2];
    L.uu = L.ux * L.ux + L.uy * L.uy + L.uz * L.uz;
    return L;
}

// LDS bytes in front of a staged kernel's other LDS data.
template <class TabT>
__device__ __forceinline__ size_t lds_table_bytes(const ApplyArgs& A, int nb) {
    return table_in_lds<TabT>() ? (((size_t)nb * A.ntab * sizeof(TabT) + 15) & ~(size_t)15) : 0;
}

template <class TabT>
__device__ __forceinline__ const TabT* stage_table(const ApplyArgs& A, int nb) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const TabT* gt = static_cast<const TabT*>(A.tab);
    if constexpr (!table_in_lds<TabT>()) return gt;
    TabT* st = reinterpret_cast<TabT*>(smem);
    const int n = nb * A.ntab;
    for (int i = threadIdx.x; i < n; i += blockDim.x) st[i] = gt[i];
    // the alignment padding after the table is zeroed (the top node's
    // neighbour in the node formats, read with weight 0)
    const int npad = (int)((lds_table_bytes<TabT>(A, nb) - (size_t)n * sizeof(TabT)) / sizeof(TabT));
    if ((int)threadIdx.x < npad) st[n + threadIdx.x] = TabT{};
    __syncthreads();
    return st;
}

// Work of one wavefront: a tile and a range of its entries.  Either every
// wavefront owns a tile (split == 0: blockDim.x/64 tiles per workgroup) or a
// workgroup owns a tile and its wavefronts split the tile's entries into
// contiguous ranges of multiples of U (split == 1).  Returns false when the
// wavefront has no tile.
__device__ __forceinline__ bool wave_work(const ApplyArgs& A, int U, int64_t& a, int64_t& eb,
                                          int64_t& ee) {
    if (A.split) {
        a = blockIdx.x;
        if (a >= A.n_act) return false;
        const int W = (int)(blockDim.x >> 6);
        const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
        const int64_t e0 = A.tptr[a], e1 = A.tptr[a + 1];
        int64_t chunk = (e1 - e0 + W - 1) / W;
        chunk = (chunk + U - 1) / U * U;
        eb = min(e1, e0 + (int64_t)wave * chunk);
        ee = min(e1, eb + chunk);
        return true;
    }
    const int t = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    a = (int64_t)__builtin_amdgcn_readfirstlane(t);
    if (a >= A.n_act) return false;
    eb = A.tptr[a];
    ee = A.tptr[a + 1];
    return true;
}

// Write one voxel value per lane; in split mode the workgroup's partial sums
// are first added in wavefront order through LDS.
template <class T>
__device__ __forceinline__ void store_voxel(const ApplyArgs& A, const LaneVox& V, T acc,
                                            T* s_acc) {
    if (A.split) {
        const int W = (int)(blockDim.x >> 6);
        const int wave = (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
        s_acc[wave * 64 + lane] = acc;
        __syncthreads();
        if (wave != 0) return;
        acc = s_acc[lane];
        for (int k = 1; k < W; ++k) acc += s_acc[k * 64 + lane];
    }
    if (V.inside) static_cast<T*>(A.out)[V.vidx] = V.act ? acc : (T)0;
}

template <class TabT>
__device__ __forceinline__ unsigned char* lds_after(const ApplyArgs& A, int nb) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    return smem + lds_table_bytes<TabT>(A, nb);
}

// Wave-uniform tile index of this wavefront (blocks hold blockDim.x/64 tiles).
__device__ __forceinline__ int64_t wave_tile() {
    const int t = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    return (int64_t)__builtin_amdgcn_readfirstlane(t);
}

// The entry lists and the per-(tile, transducer) constants are read-only in
// every kernel that reads them.  Loading them through the constant address
// space states it, so these wave-uniform loads stay on the scalar path also in
// the J kernels, whose stores inside the entry loop would otherwise turn them
// into vector loads followed by readfirstlane.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
using ConstU4 = const __attribute__((address_space(4))) u32x4;
using ConstU2 = const __attribute__((address_space(4))) u32x2;
__device__ __forceinline__ Entry entry_at(const Entry* ents, int64_t e) {
    return __builtin_bit_cast(Entry, ((ConstU4*)(ents + e))[0]);
}
__device__ __forceinline__ TxConst tx_at(const TxConst* row, int q) {
    struct Words { u32x2 w[5]; } v;
    static_assert(sizeof(Words) == sizeof(TxConst), "TxConst words");
    ConstU2* p = (ConstU2*)(row + q);
#pragma unroll
    for (int k = 0; k < 5; ++k) v.w[k] = p[k];
    return __builtin_bit_cast(TxConst, v);
}

// Source part of U consecutive entries: recomputed only when the source
// changes (entries are sorted by source, receiver within a tile).
template <int U, class F, class Dist>
__device__ __forceinline__ void source_parts(const Entry (&E)[U], const TxConst* row,
                                             const LaneVox& V, int& prev, F& ds, F& as,
                                             F (&dsu)[U], F (&asu)[U], Dist dist) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int s = (int)(E[u].sr & 0xffffu);
        if (s != prev) {
            prev = s;
            dist(tx_at(row, s), V.ux, V.uy, V.uz, V.uu, ds, as);
        }
        dsu[u] = ds;
        asu[u] = as;
    }
}

// J^T, FP32 / BF16 table: dc_j = sum_i sum_b J^b_ij dT^b_i.
template <int NB, class TabT, int U>
__device__ __forceinline__ void jt32_step(const ApplyArgs& A, const TabT* st,
                                          const Entry* __restrict__ ents,
                                          const TxConst* __restrict__ row,
                                          const float* __restrict__ w, const LaneVox& V,
                                          float nm1, int64_t e, int& prev, float& ds, float& rss,
                                          float& acc) {
    Entry E[U];
#pragma unroll
    for (int u = 0; u < U; ++u) E[u] = entry_at(ents, e + u);
    float wu[U][NB];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int b = 0; b < NB; ++b) wu[u][b] = w[b * A.M + E[u].p];
    float dsu[U], rssu[U], dr[U], rsr[U];
    source_parts<U>(E, row, V, prev, ds, rss, dsu, rssu, dist32);
#pragma unroll
    for (int u = 0; u < U; ++u) dist32(tx_at(row, (int)(E[u].sr >> 16)), V.ux, V.uy, V.uz, V.uu, dr[u], rsr[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const float R = (dsu[u] + dr[u]) + E[u].R0hi;
        float hw = 0.f;
#pragma unroll
        for (int b = 0; b < NB; ++b)
            hw = fmaf(lookup(st + b * A.ntab, R, A.inv_dr[b], nm1), wu[u][b], hw);
        acc = fmaf(hw, rssu[u] * rsr[u], acc);
    }
}

template <int NB, class TabT, int U>
__global__ __launch_bounds__(1024) void k_jt32(ApplyArgs A) {
    const TabT* st = stage_table<TabT>(A, NB);
    float* s_acc = reinterpret_cast<float*>(lds_after<TabT>(A, NB));
    int64_t a, e0, e1;
    if (!wave_work(A, U, a, e0, e1)) return;
    const int lane = threadIdx.x & 63;
    const LaneVox V = lane_vox(A, a, lane);
    const TxConst* __restrict__ row = A.txc + a * A.n_tx;
    const float* __restrict__ w = static_cast<const float*>(A.w);
    const float nm1 = (float)(A.ntab - 1);
    float acc = 0.f, ds = 0.f, rss = 0.f;
    int prev = -1;
    int64_t e = e0;
    for (; e + U <= e1; e += U) jt32_step<NB, TabT, U>(A, st, A.ents, row, w, V, nm1, e, prev, ds, rss, acc);
    for (; e < e1; ++e) jt32_step<NB, TabT, 1>(A, st, A.ents, row, w, V, nm1, e, prev, ds, rss, acc);
    store_voxel(A, V, acc, s_acc);
}

// J, FP32 / BF16 table: partial[b][e] = sum_{j in tile} h^b(R_ij) A_ij / C_i dc_j.
// The U entries of a step are reduced together; lane u then stores entry e+u.
template <int NB, class TabT, int U>
__device__ __forceinline__ void j32_step(const ApplyArgs& A, const TabT* st,
                                         const Entry* __restrict__ ents,
                                         const TxConst* __restrict__ row, float* __restrict__ part,
                                         const LaneVox& V, float xv, float nm1, int lane, int64_t e,
                                         int& prev, float& ds, float& rss) {
    Entry E[U];
#pragma unroll
    for (int u = 0; u < U; ++u) E[u] = entry_at(ents, e + u);
    float dsu[U], rssu[U], dr[U], rsr[U];
    source_parts<U>(E, row, V, prev, ds, rss, dsu, rssu, dist32);
#pragma unroll
    for (int u = 0; u < U; ++u) dist32(tx_at(row, (int)(E[u].sr >> 16)), V.ux, V.uy, V.uz, V.uu, dr[u], rsr[u]);
    float R[U], t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        R[u] = (dsu[u] + dr[u]) + E[u].R0hi;
        t[u] = (rssu[u] * xv) * rsr[u];
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = lookup(st + b * A.ntab, R[u], A.inv_dr[b], nm1) * t[u];
        const float sum = multi_sum<U>(v, lane);
        if (lane < U) part[b * A.nnz + e + lane] = sum;
    }
}

template <int NB, class TabT, int U>
__global__ __launch_bounds__(1024) void k_j32(ApplyArgs A) {
    const TabT* st = stage_table<TabT>(A, NB);
    int64_t a, e0, e1;
    if (!wave_work(A, U, a, e0, e1)) return;
    const int lane = threadIdx.x & 63;
    const LaneVox V = lane_vox(A, a, lane);
    const TxConst* __restrict__ row = A.txc + a * A.n_tx;
    float* __restrict__ part = static_cast<float*>(A.out);
    const float xv = V.act ? static_cast<const float*>(A.x)[A.nxy ? V.vidx % A.nxy : V.vidx] : 0.f;
    const float nm1 = (float)(A.ntab - 1);
    float ds = 0.f, rss = 0.f;
    int prev = -1;
    int64_t e = e0;
    for (; e + U <= e1; e += U)
        j32_step<NB, TabT, U>(A, st, A.ents, row, part, V, xv, nm1, lane, e, prev, ds, rss);
    for (; e < e1; ++e)
        j32_step<NB, TabT, 1>(A, st, A.ents, row, part, V, xv, nm1, lane, e, prev, ds, rss);
}

// FP64 counterparts.
template <int NB, int U>
__device__ __forceinline__ void jt64_step(const ApplyArgs& A, const double2* st,
                                          const Entry* __restrict__ ents,
                                          const TxConst* __restrict__ row,
                                          const double* __restrict__ w, const LaneVox& V,
                                          double nm1, int64_t e, int& prev, double& ds,
                                          double& gs, double& acc) {
    Entry E[U];
#pragma unroll
    for (int u = 0; u < U; ++u) E[u] = entry_at(ents, e + u);
    double dsu[U], gsu[U], dr[U], gr[U];
    source_parts<U>(E, row, V, prev, ds, gs, dsu, gsu, dist64);
#pragma unroll
    for (int u = 0; u < U; ++u) dist64(tx_at(row, (int)(E[u].sr >> 16)), V.ux, V.uy, V.uz, V.uu, dr[u], gr[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const double R = (dsu[u] + dr[u]) + ((double)E[u].R0hi + (double)E[u].R0lo);
        double hw = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b)
            hw = fma(lookup(st + b * A.ntab, R, A.inv_dr64[b], nm1), w[b * A.M + E[u].p], hw);
        acc = fma(hw, gsu[u] * gr[u], acc);
    }
}

template <int NB, bool LDS_TAB, int U>
__global__ __launch_bounds__(1024) void k_jt64(ApplyArgs A) {
    const double2* st = LDS_TAB ? stage_table<double2>(A, NB) : static_cast<const double2*>(A.tab);
    double* s_acc = reinterpret_cast<double*>(lds_after<double2>(A, LDS_TAB ? NB : 0));
    int64_t a, e0, e1;
    if (!wave_work(A, U, a, e0, e1)) return;
    const int lane = threadIdx.x & 63;
    const LaneVox V = lane_vox(A, a, lane);
    const TxConst* __restrict__ row = A.txc + a * A.n_tx;
    const double* __restrict__ w = static_cast<const double*>(A.w);
    const double nm1 = (double)(A.ntab - 1);
    double acc = 0.0, ds = 0.0, gs = 0.0;
    int prev = -1;
    int64_t e = e0;
    for (; e + U <= e1; e += U) jt64_step<NB, U>(A, st, A.ents, row, w, V, nm1, e, prev, ds, gs, acc);
    for (; e < e1; ++e) jt64_step<NB, 1>(A, st, A.ents, row, w, V, nm1, e, prev, ds, gs, acc);
    store_voxel(A, V, acc, s_acc);
}

template <int NB, int U>
__device__ __forceinline__ void j64_step(const ApplyArgs& A, const double2* st,
                                         const Entry* __restrict__ ents,
                                         const TxConst* __restrict__ row,
                                         double* __restrict__ part, const LaneVox& V, double xv,
                                         double nm1, int lane, int64_t e, int& prev, double& ds,
                                         double& gs) {
    Entry E[U];
#pragma unroll
    for (int u = 0; u < U; ++u) E[u] = entry_at(ents, e + u);
    double dsu[U], gsu[U], dr[U], gr[U];
    source_parts<U>(E, row, V, prev, ds, gs, dsu, gsu, dist64);
#pragma unroll
    for (int u = 0; u < U; ++u) dist64(tx_at(row, (int)(E[u].sr >> 16)), V.ux, V.uy, V.uz, V.uu, dr[u], gr[u]);
    double R[U], t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        R[u] = (dsu[u] + dr[u]) + ((double)E[u].R0hi + (double)E[u].R0lo);
        t[u] = (gsu[u] * xv) * gr[u];
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = lookup(st + b * A.ntab, R[u], A.inv_dr64[b], nm1) * t[u];
        const double sum = multi_sum<U>(v, lane);
        if (lane < U) part[b * A.nnz + e + lane] = sum;
    }
}

template <int NB, bool LDS_TAB, int U>
__global__ __launch_bounds__(1024) void k_j64(ApplyArgs A) {
    const double2* st = LDS_TAB ? stage_table<double2>(A, NB) : static_cast<const double2*>(A.tab);
    int64_t a, e0, e1;
    if (!wave_work(A, U, a, e0, e1)) return;
    const int lane = threadIdx.x & 63;
    const LaneVox V = lane_vox(A, a, lane);
    const TxConst* __restrict__ row = A.txc + a * A.n_tx;
    double* __restrict__ part = static_cast<double*>(A.out);
    const double xv = V.act ? static_cast<const double*>(A.x)[A.nxy ? V.vidx % A.nxy : V.vidx] : 0.0;
    const double nm1 = (double)(A.ntab - 1);
    double ds = 0.0, gs = 0.0;
    int prev = -1;
    int64_t e = e0;
    for (; e + U <= e1; e += U)
        j64_step<NB, U>(A, st, A.ents, row, part, V, xv, nm1, lane, e, prev, ds, gs);
    for (; e < e1; ++e)
        j64_step<NB, 1>(A, st, A.ents, row, part, V, xv, nm1, lane, e, prev, ds, gs);
}

// One wavefront per tile, waves_per_block tiles per workgroup sharing the
// LDS copy of the tables.
template <class K>
static hipError_t launch_k(K kern, hipStream_t s, const ApplyArgs& a, size_t table_bytes,
                           size_t acc_bytes) {
    if (a.n_act == 0) return hipSuccess;
    const int wpb = a.waves_per_block;
    const size_t lds = ((table_bytes + 15) & ~(size_t)15) + (a.split ? acc_bytes * 64 * wpb : 0);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const unsigned nblk = a.split ? (unsigned)a.n_act : (unsigned)((a.n_act + wpb - 1) / wpb);
    hipLaunchKernelGGL(kern, dim3(nblk), dim3(64 * wpb), lds, s, a);
    return hipGetLastError();
}

template <int NB, int U>
static hipError_t launch_nbu(hipStream_t s, fftt_precision prec, bool transpose,
                             const ApplyArgs& a) {
    const size_t n = (size_t)NB * a.ntab;
    switch (prec) {
        case FFTT_FP32:
            return transpose ? launch_k(k_jt32<NB, float2, U>, s, a, n * sizeof(float2), 4)
                             : launch_k(k_j32<NB, float2, U>, s, a, n * sizeof(float2), 0);
        case FFTT_FP32_BF16TABLE:
            return transpose ? launch_k(k_jt32<NB, uint32_t, U>, s, a, n * sizeof(uint32_t), 4)
                             : launch_k(k_j32<NB, uint32_t, U>, s, a, n * sizeof(uint32_t), 0);
        case FFTT_FP64: {
            const size_t bytes = n * sizeof(double2);
            if (bytes <= 131072)
                return transpose ? launch_k(k_jt64<NB, true, U>, s, a, bytes, 8)
                                 : launch_k(k_j64<NB, true, U>, s, a, bytes, 0);
            return transpose ? launch_k(k_jt64<NB, false, U>, s, a, 0, 8)
                             : launch_k(k_j64<NB, false, U>, s, a, 0, 0);
        }
    }
    return hipErrorInvalidValue;
}

template <int NB>
static hipError_t launch_nb(hipStream_t s, fftt_precision prec, bool transpose,
                            const ApplyArgs& a) {
    switch (a.unroll) {
        case 1: return launch_nbu<NB, 1>(s, prec, transpose, a);
        case 2: return launch_nbu<NB, 2>(s, prec, transpose, a);
        case 4: return launch_nbu<NB, 4>(s, prec, transpose, a);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_apply(hipStream_t s, fftt_precision prec, bool transpose, const ApplyArgs& a) {
    switch (a.nb) {
        case 1: return launch_nb<1>(s, prec, transpose, a);
        case 2: return launch_nb<2>(s, prec, transpose, a);
        case 3: return launch_nb<3>(s, prec, transpose, a);
        case 4: return launch_nb<4>(s, prec, transpose, a);
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------ staged (separable) kernels
//
// A workgroup owns one tile.  First its wavefronts evaluate, for every lane
// (voxel) and every transducer q, delta_q = R_xq - D0f_q and 1/R_xq once and
// keep them in LDS ([q][lane] float2).  A pair (s, r) then needs only two LDS
// reads: R = R0 + delta_s + delta_r, A ~ (1/R_xs)(1/R_xr).  The tile's pair
// list is split over the wavefronts in contiguous ranges of multiples of U.
// Used when the tables plus n_tx * 512 bytes fit in LDS.

template <class TabT>
__device__ __forceinline__ float2* staged_tx(const ApplyArgs& A, int nb) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    return reinterpret_cast<float2*>(smem + lds_table_bytes<TabT>(A, nb));
}

// Stages transducers q0 .. q0 + n - 1 into sx[q - q0][lane].
// With the FP32 constants (A.txc32) n is formed in FP32 (see TxConst32);
// c: the six words of a TxConst32.
__device__ __forceinline__ void dist32f(const float (&c)[6], float ux, float uy, float uz,
                                        float uu, float& delta, float& rs) {
    const float n = fmaf(c[0], ux, fmaf(c[1], uy, fmaf(c[2], uz, uu + c[3])));
    const float q = c[5] + n;
    rs = __builtin_amdgcn_rsqf(q);
    delta = n * __builtin_amdgcn_rcpf(q * rs + c[4]);
}

__device__ __forceinline__ void stage_distances(const ApplyArgs& A, int64_t a, const LaneVox& V,
                                                float2* sx, int lane, int q0, int n) {
    const int W = (int)(blockDim.x >> 6);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    ConstF* row = (ConstF*)(A.txc32 + a * A.n_tx + q0);
    const float ux = (float)V.ux, uy = (float)V.uy, uz = (float)V.uz, uu = (float)V.uu;
    int q = wave;
    // four transducers per step: their constants are requested together
    for (; q + 3 * W < n; q += 4 * W) {
        float c[4][6];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int j = 0; j < 6; ++j) c[k][j] = row[6 * (q + k * W) + j];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float d, rs;
            dist32f(c[k], ux, uy, uz, uu, d, rs);
            sx[(q + k * W) * 64 + lane] = make_float2(d * A.inv_dr[0], rs);
        }
    }
    for (; q < n; q += W) {
        float c[6], d, rs;
#pragma unroll
        for (int j = 0; j < 6; ++j) c[j] = row[6 * q + j];
        dist32f(c, ux, uy, uz, uu, d, rs);
        sx[q * 64 + lane] = make_float2(d * A.inv_dr[0], rs);
    }
    __syncthreads();
}

// Entries of one step, loaded as whole 16-byte records (one scalar batch).
template <int U>
struct StepEntries {
    int p[U];
    int s[U];
    int r[U];
    float R0[U];
    int m[U];   // the staged copies: bands whose kernel can be nonzero (else all)
};

// Transducer indices are returned relative to the staged block's first one.
// The entries are read through the constant address space (see entry_at).

template <int U>
__device__ __forceinline__ StepEntries<U> load_entries(const Entry* __restrict__ ents, int64_t e,
                                                       int base) {
    StepEntries<U> E;
    ConstU4* raw = (ConstU4*)(ents + e);
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = raw[u];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        E.p[u] = (int)v[u].x;
        E.s[u] = (int)(v[u].y & 0xffffu) - base;
        E.r[u] = (int)(v[u].y >> 16) - base;
        E.R0[u] = __uint_as_float(v[u].z);
        E.m[u] = 0xf;
    }
    return E;
}

// The staged J's entries: (sr, R0hi) word pairs, eight bytes each (the pair
// index is not needed there); StepEntries.p is left unset.  The copies' sr
// word is s | r << 14 | bands << 28.
template <int U>
__device__ __forceinline__ StepEntries<U> load_entries(const uint32_t* __restrict__ ents8,
                                                       int64_t e, int base) {
    StepEntries<U> E;
    ConstU2* raw = (ConstU2*)(ents8 + 2 * e);
    u32x2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = raw[u];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        E.p[u] = 0;
        E.s[u] = (int)(v[u].x & 0x3fffu) - base;
        E.r[u] = (int)((v[u].x >> 14) & 0x3fffu) - base;
        E.R0[u] = __uint_as_float(v[u].y);
        E.m[u] = (int)(v[u].x >> 28);
    }
    return E;
}

// The staged J^T's entries: (p, sr, R0hi), twelve bytes each.
using ConstU1 = const __attribute__((address_space(4))) uint32_t;
template <int U>
__device__ __forceinline__ StepEntries<U> load_entries(const Entry3* __restrict__ ents3,
                                                       int64_t e, int base) {
    StepEntries<U> E;
    ConstU1* raw = (ConstU1*)(ents3 + e);
    uint32_t v[3 * U];
#pragma unroll
    for (int i = 0; i < 3 * U; ++i) v[i] = raw[i];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        E.p[u] = (int)v[3 * u];
        E.s[u] = (int)(v[3 * u + 1] & 0x3fffu) - base;
        E.r[u] = (int)((v[3 * u + 1] >> 14) & 0x3fffu) - base;
        E.R0[u] = __uint_as_float(v[3 * u + 2]);
        E.m[u] = (int)(v[3 * u + 1] >> 28);
    }
    return E;
}

// A float in the global address space (for pointers rebuilt from integers,
// which would otherwise be generic and take flat instructions).
typedef __attribute__((address_space(1))) float GlobalF;

__device__ __forceinline__ int64_t uniform64(int64_t x) {
    const uint64_t u = (uint64_t)x;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Transducer blocks of the staged kernels: aligned index ranges
// [b Q, b Q + Q).  Every kernel pair lies in one block (checked on the host)
// and a tile's entries are sorted by source, so they form one run per block;
// the workgroup stages one block at a time.  First entry in [e, t1) whose
// source is at least q (uniform binary search).
__device__ __forceinline__ int source_at(const Entry* __restrict__ ents, int64_t e) {
    return (int)(ents[e].sr & 0xffffu);
}
__device__ __forceinline__ int source_at(const uint32_t* __restrict__ ents8, int64_t e) {
    return (int)(ents8[2 * e] & 0x3fffu);
}
__device__ __forceinline__ int source_at(const Entry3* __restrict__ ents3, int64_t e) {
    return (int)(ents3[e].sr & 0x3fffu);
}
template <class EntT>
__device__ __forceinline__ int64_t first_source_at_least(const EntT* __restrict__ ents,
                                                        int64_t e, int64_t t1, int q) {
    int64_t lo = e, hi = t1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (source_at(ents, mid) < q)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Runs body(q0, e0, e1) for each transducer block of tile a after staging
// it; e0 .. e1 is this wavefront's share of the block's entries (multiples of
// U).  The staged values are valid inside body only.
template <int U, class EntT, class F>
__device__ __forceinline__ void for_each_block(const ApplyArgs& A, const EntT* ents,
                                               const int64_t* tptr, int64_t a, float2* sx,
                                               int lane, F&& body) {
    const int Q = A.stage_q;
    const int W = (int)(blockDim.x >> 6);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t t0 = tptr[a], t1 = tptr[a + 1];
    for (int64_t b0 = t0; b0 < t1;) {
        const int q0 = source_at(ents, b0) / Q * Q;
        // usually one block holds all of the tile's remaining entries
        const int64_t b1 = source_at(ents, t1 - 1) < q0 + Q
                               ? t1
                               : first_source_at_least(ents, b0, t1, q0 + Q);
        // the lane's voxel offsets are recomputed per block rather than kept
        // live through the entry loop
        stage_distances(A, a, lane_vox(A, a, lane), sx, lane, q0, min(Q, (int)A.n_tx - q0));
        int64_t chunk = (b1 - b0 + W - 1) / W;
        chunk = (chunk + U - 1) / U * U;
        const int64_t e0 = min(b1, b0 + (int64_t)wave * chunk);
        const int64_t e1 = min(b1, e0 + chunk);
        // wave-uniform by construction; stated so that the entries are read
        // with scalar loads and handled by scalar instructions
        body(__builtin_amdgcn_readfirstlane(q0), uniform64(e0), uniform64(e1));
        __syncthreads();   // before the next block is staged over this one
        b0 = b1;
    }
}

// Source terms of a J^T step: the scaled detour part and 1/R_xs.  The last
// source read is cached (prev, cd, cg); a step whose entries share one source
// needs one LDS read at most (none when it is the cached one), any other step
// reads every entry's source.  A step of eight is taken as two halves of four
// that are handled so: J^T walks source-grouped lists on which almost every
// half shares its source.  The arithmetic of the step is instantiated per
// case so that shared values are used in place (no register copies); an
// empty asm statement, distinct per case, ends each case so that the
// compiler does not merge their arithmetic into one block (which brings the
// copies back: up to 14 v_mov per step).  body also receives, as a
// compile-time constant, which entries share one source: bit 0 the first
// half of the step, bit 1 the second half, bit 2 all of it.
template <int U, class F>
__device__ __forceinline__ void with_sources(const StepEntries<U>& E, const float2* sx, int lane,
                                             int& prev, float& cd, float& cg, F&& body) {
    auto fetch = [&](int q, float& d, float& g) {
        const float2 v = sx[q * 64 + lane];
        d = v.x;
        g = v.y;
    };
    auto refresh = [&](int q) {
        if (q != prev) {
            fetch(q, cd, cg);
            prev = q;
        }
    };
    if constexpr (U == 8) {
        bool lo = true, hi = true;
#pragma unroll
        for (int u = 1; u < 4; ++u) lo = lo && (E.s[u] == E.s[0]);
#pragma unroll
        for (int u = 5; u < 8; ++u) hi = hi && (E.s[u] == E.s[4]);
        float d[8], g[8];
        if (lo && hi) {
            refresh(E.s[0]);
            if (E.s[4] == E.s[0]) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    d[u] = cd;
                    g[u] = cg;
                }
                body(d, g, std::integral_constant<int, 7>{});
                asm volatile("; source case 1");
            } else {
                float hd, hg;
                fetch(E.s[4], hd, hg);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    d[u] = cd;
                    g[u] = cg;
                    d[u + 4] = hd;
                    g[u + 4] = hg;
                }
                body(d, g, std::integral_constant<int, 3>{});
                asm volatile("; source case 2");
                prev = E.s[4];
                cd = hd;
                cg = hg;
            }
        } else if (lo) {
            refresh(E.s[0]);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                d[u] = cd;
                g[u] = cg;
                fetch(E.s[u + 4], d[u + 4], g[u + 4]);
            }
            body(d, g, std::integral_constant<int, 1>{});
            asm volatile("; source case 3");
            prev = E.s[7];
            cd = d[7];
            cg = g[7];
        } else if (hi) {
#pragma unroll
            for (int u = 0; u < 4; ++u) fetch(E.s[u], d[u], g[u]);
            refresh(E.s[4]);
#pragma unroll
            for (int u = 4; u < 8; ++u) {
                d[u] = cd;
                g[u] = cg;
            }
            body(d, g, std::integral_constant<int, 2>{});
            asm volatile("; source case 4");
        } else {
#pragma unroll
            for (int u = 0; u < 8; ++u) fetch(E.s[u], d[u], g[u]);
            body(d, g, std::integral_constant<int, 0>{});
            asm volatile("; source case 5");
            prev = E.s[7];
            cd = d[7];
            cg = g[7];
        }
        return;
    }
    bool same = true;
#pragma unroll
    for (int u = 1; u < U; ++u) same = same && (E.s[u] == E.s[0]);
    float d[U], g[U];
    if (same) {
        refresh(E.s[0]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            d[u] = cd;
            g[u] = cg;
        }
        body(d, g, std::integral_constant<int, 7>{});
        asm volatile("; source case 6");
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u) fetch(E.s[u], d[u], g[u]);
        body(d, g, std::integral_constant<int, 0>{});
        asm volatile("; source case 7");
        prev = E.s[U - 1];
        cd = d[U - 1];
        cg = g[U - 1];
    }
}

template <int NB, int U>
struct StepWeights {
    float w[U][NB];
};

// The weights of a step go through the vector memory path: the pair's byte
// offset is copied into a VGPR by one v_mov (written as asm, so the compiler
// cannot see that the value is wave-uniform and fold the loads back into
// scalar loads), so the loads are counted by vmcnt and their latency overlaps
// the step's LDS reads instead of adding a second dependent scalar-memory
// round trip after the entries.
__device__ __forceinline__ uint32_t to_vgpr(uint32_t x) {
    uint32_t v;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(x));
    return v;
}
template <int NB, int U>
__device__ __forceinline__ StepWeights<NB, U> load_weights(const ApplyArgs& A,
                                                          const float* __restrict__ w,
                                                          const StepEntries<U>& E) {
    StepWeights<NB, U> W;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        // 32-bit byte offset, scaled on the scalar side; the band's base stays
        // in scalar registers
        const uint32_t off = to_vgpr((uint32_t)E.p[u] << 2);
#pragma unroll
        for (int b = 0; b < NB; ++b)
            W.w[u][b] = *reinterpret_cast<const float*>(
                reinterpret_cast<const char*>(w + (size_t)b * A.M) + off);
    }
    return W;
}

// MODE of the J^T kernel: 0 = J^T dT (weights C_p sum dT); 1 = sensitivity
// coverage sum_i |J_ij| (weights |C_p| m_p, |h|); 2 = diag(J^T J) =
// sum_i J_ij^2 (weights C_p^2 m_p, h^2, (1/(R_xs R_xr))^2); m_p = caller
// pairs sharing kernel pair p.
template <int NB, class TabT, int U, int MODE = 0>
__device__ __forceinline__ void jt32s_body(const ApplyArgs& A, const TabT* st, const float2* sx,
                                           const StepEntries<U>& E, const StepWeights<NB, U>& W,
                                           float nm1, int lane, int& prev, float& cd, float& cg,
                                           float& acc) {
    float rd[U], rg[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const float2 v = sx[E.r[u] * 64 + lane];
        rd[u] = v.x;
        rg[u] = v.y;
    }
    // one band: the pair weight goes into the receiver factor as soon as it
    // arrives (fewer live registers over the lookups than h w formed after)
    constexpr bool WR = NB == 1 && MODE != 2;
    if constexpr (WR) {
#pragma unroll
        for (int u = 0; u < U; ++u) rg[u] *= W.w[u][0];
    }
    with_sources<U>(E, sx, lane, prev, cd, cg,
                    [&](const float (&sd)[U], const float (&sg)[U], auto share) {
        constexpr int SH = decltype(share)::value;
        float x0[U], hw[U];
#pragma unroll
        for (int u = 0; u < U; ++u)   // R / dR_0 = (delta_s + delta_r) / dR_0 + R0 / dR_0
            x0[u] = fmaf(E.R0[u], A.inv_dr[0], sd[u] + rd[u]);
        // bands whose kernel is zero for every entry of the step are skipped
        int bands = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) bands |= E.m[u];
        if constexpr (NB > 1) {
#pragma unroll
            for (int u = 0; u < U; ++u) hw[u] = 0.0f;
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (NB > 1 && !((bands >> b) & 1)) continue;
            float xb[U], h[U];
#pragma unroll
            for (int u = 0; u < U; ++u) xb[u] = b == 0 ? x0[u] : x0[u] * A.xr[b];
            lookup_n<U>(band_tab(st, b, A.ntab), xb, nm1, h);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if constexpr (MODE == 1) h[u] = fabsf(h[u]);
                if constexpr (MODE == 2) h[u] *= h[u];
                hw[u] = WR ? h[u] : (NB == 1 ? h[u] * W.w[u][0] : fmaf(h[u], W.w[u][b], hw[u]));
            }
        }
        // sum_u hw_u / (R_xs R_xr) (one band: w_u already in the 1/R_xr
        // factor): entries that share a source add sum_u hw_u / R_xr first
        // and take 1/R_xs once
        auto shared = [&](int u0, int u1) {
            float t = hw[u0] * rg[u0];
#pragma unroll
            for (int u = u0 + 1; u < u1; ++u) t = fmaf(hw[u], rg[u], t);
            acc = fmaf(t, sg[u0], acc);
        };
        auto each = [&](int u0, int u1) {
#pragma unroll
            for (int u = u0; u < u1; ++u) {
                const float g = sg[u] * rg[u];
                acc = fmaf(hw[u], MODE == 2 ? g * g : g, acc);
            }
        };
        if constexpr (MODE == 2) {
            each(0, U);
        } else if constexpr ((SH & 4) != 0) {
            shared(0, U);
        } else {
            if constexpr ((SH & 1) != 0) shared(0, U / 2); else each(0, U / 2);
            if constexpr ((SH & 2) != 0) shared(U / 2, U); else each(U / 2, U);
        }
    });
}

template <int NB, class TabT, int U, int MODE = 0>
__global__ __launch_bounds__(1024, NB == 1 ? 8 : 4) void k_jt32s(ApplyArgs A) {
    const TabT* st = stage_table<TabT>(A, NB);
    float2* sx = staged_tx<TabT>(A, NB);
    const int64_t a = blockIdx.x;
    if (a >= A.n_act) return;
    const int lane = threadIdx.x & 63;
    const float* __restrict__ w = static_cast<const float*>(A.w);
    const float nm1 = (float)(A.ntab - 1);
    float acc = 0.f;
    // J^T walks its own copy of the lists; the coverage passes the originals
    const auto* ents = MODE == 0 ? (const void*)A.ents3 : (const void*)A.ents;
    using EntT = std::conditional_t<MODE == 0, Entry3, Entry>;
    const EntT* el = static_cast<const EntT*>(ents);
    for_each_block<U>(A, el, MODE == 0 ? A.tptr3 : A.tptr, a, sx, lane,
                      [&](int q0, int64_t e0, int64_t e1) {
        float cd = 0.f, cg = 0.f;
        int prev = -1;
        int64_t e = e0;
        // a 32-bit step count keeps the loop test on the scalar unit
        for (int n = (int)((e1 - e0) / U); n > 0; --n, e += U) {
            const StepEntries<U> E = load_entries<U>(el, e, q0);
            jt32s_body<NB, TabT, U, MODE>(A, st, sx, E, load_weights<NB, U>(A, w, E), nm1, lane,
                                          prev, cd, cg, acc);
        }
        for (; e < e1; ++e) {
            const StepEntries<1> E = load_entries<1>(el, e, q0);
            jt32s_body<NB, TabT, 1, MODE>(A, st, sx, E, load_weights<NB, 1>(A, w, E), nm1, lane,
                                          prev, cd, cg, acc);
        }
    });
    // combine the wavefronts in order (the staged distances are no longer
    // needed; the block loop ended with a barrier)
    float* s_acc = reinterpret_cast<float*>(sx);
    const int wave = (int)(threadIdx.x >> 6);
    s_acc[wave * 64 + lane] = acc;
    __syncthreads();
    if (wave != 0) return;
    const int W = (int)(blockDim.x >> 6);
    float t = s_acc[lane];
    for (int k = 1; k < W; ++k) t += s_acc[k * 64 + lane];
    bool inside, act;
    int64_t vidx, v[3];
    voxel_of_lane(A, a, lane, inside, act, vidx, v);
    if (inside) static_cast<float*>(A.out)[vidx] = act ? t : 0.f;
}

// Source terms of a J step: the scaled detour part and dc_j / R_xs.  J walks
// the lists in pair order, in which a tile's entries of one source form runs
// (about 13 entries on average for a 128-element ring): a step inside one run
// reads its source once, any other step reads every entry's source.  Nothing
// is kept from one step to the next (a cached source costs register copies
// at every step; so did instantiating the arithmetic for each split point of
// a step over two runs, which was slower overall).
template <int U, class F>
__device__ __forceinline__ void with_sources_j(const StepEntries<U>& E, const float2* sx,
                                               int lane, float factor, F&& body) {
    auto fetch = [&](int q, float& d, float& g) {
        const float2 v = sx[q * 64 + lane];
        d = v.x;
        g = v.y * factor;
    };
    float d[U], g[U];
    bool same = true;
#pragma unroll
    for (int u = 1; u < U; ++u) same = same && (E.s[u] == E.s[0]);
    if (same) {
        float a, ga;
        fetch(E.s[0], a, ga);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            d[u] = a;
            g[u] = ga;
        }
        body(d, g);
        asm volatile("; J sources: one run");
        return;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) fetch(E.s[u], d[u], g[u]);
    body(d, g);
    asm volatile("; J sources: per entry");
}

template <int NB, class TabT, int U>
__device__ __forceinline__ void j32s_body(const ApplyArgs& A, const TabT* st, const float2* sx,
                                          const StepEntries<U>& E, float* __restrict__ part,
                                          float xv, float nm1, int lane, int64_t e) {
    float rd[U], rg[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const float2 v = sx[E.r[u] * 64 + lane];
        rd[u] = v.x;
        rg[u] = v.y;
    }
    // source factor dc_j / R_xs
    with_sources_j<U>(E, sx, lane, xv, [&](const float (&sd)[U], const float (&sg)[U]) {
        float x0[U], t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            x0[u] = fmaf(E.R0[u], A.inv_dr[0], sd[u] + rd[u]);
            t[u] = sg[u] * rg[u];
        }
        // bands whose kernel is zero for every entry of the step: zero sums
        int bands = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) bands |= E.m[u];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            float sum = 0.0f;
            if (NB == 1 || ((bands >> b) & 1)) {
                float xb[U], v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) xb[u] = b == 0 ? x0[u] : x0[u] * A.xr[b];
                lookup_n<U>(band_tab(st, b, A.ntab), xb, nm1, v);
#pragma unroll
                for (int u = 0; u < U; ++u) v[u] *= t[u];
                sum = multi_sum<U>(v, lane);
            }
            // uniform base, per-lane 32-bit offset (scalar-base stores; the
            // base is passed through readfirstlane so that it is not folded
            // into a per-lane pointer advanced by a vector add each step)
            GlobalF* pe = reinterpret_cast<GlobalF*>(
                uniform64(reinterpret_cast<int64_t>(part + (b * A.nnz + e))));
            if constexpr (U == 8) {
                if ((lane & 7) == 0) pe[sum8_value_of_lane(lane)] = sum;
            } else {
                if (lane < U) pe[lane] = sum;
            }
        }
    });
}

template <int NB, class TabT, int U>
__global__ __launch_bounds__(1024, NB == 1 ? 8 : 4) void k_j32s(ApplyArgs A) {
    const TabT* st = stage_table<TabT>(A, NB);
    float2* sx = staged_tx<TabT>(A, NB);
    const int64_t a = blockIdx.x;
    if (a >= A.n_act) return;
    const int lane = threadIdx.x & 63;
    float* __restrict__ part = static_cast<float*>(A.out);
    float xv;
    {
        bool inside, act;
        int64_t vidx, v[3];
        voxel_of_lane(A, a, lane, inside, act, vidx, v);
        xv = act ? static_cast<const float*>(A.x)[A.nxy ? v[0] + A.g.dims[0] * v[1] : vidx] : 0.f;
    }
    const float nm1 = (float)(A.ntab - 1);
    for_each_block<U>(A, A.ents8, A.tptr, a, sx, lane, [&](int q0, int64_t e0, int64_t e1) {
        int64_t e = e0;
        // a 32-bit step count keeps the loop test on the scalar unit
        for (int n = (int)((e1 - e0) / U); n > 0; --n, e += U)
            j32s_body<NB, TabT, U>(A, st, sx, load_entries<U>(A.ents8, e, q0), part, xv, nm1,
                                   lane, e);
        for (; e < e1; ++e)
            j32s_body<NB, TabT, 1>(A, st, sx, load_entries<1>(A.ents8, e, q0), part, xv, nm1,
                                   lane, e);
    });
}

template <class K>
static hipError_t launch_staged(K kern, hipStream_t s, const ApplyArgs& a, size_t table_bytes) {
    if (a.n_act == 0) return hipSuccess;
    const int wpb = a.waves_per_block;
    const size_t tx_bytes = std::max<size_t>((size_t)a.stage_q * 64 * sizeof(float2),
                                             (size_t)wpb * 64 * sizeof(float));
    const size_t lds = ((table_bytes + 15) & ~(size_t)15) + tx_bytes;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)a.n_act), dim3(64 * wpb), lds, s, a);
    return hipGetLastError();
}

static size_t staged_entry_bytes(int tabfmt) {
    return tabfmt == STAB_PAIR32 ? sizeof(float2) : tabfmt == STAB_SERIES ? 0 : sizeof(float);
}

size_t staged_lds_bytes(int nb, int ntab, int tabfmt, int64_t q, int wpb) {
    const size_t tab = (size_t)nb * ntab * staged_entry_bytes(tabfmt);
    return ((tab + 15) & ~(size_t)15) +
           std::max<size_t>((size_t)q * 64 * sizeof(float2), (size_t)wpb * 64 * sizeof(float));
}

template <class TabT, int NB, int U>
static hipError_t launch_staged_t(hipStream_t s, bool transpose, const ApplyArgs& a) {
    const size_t bytes = table_in_lds<TabT>() ? (size_t)NB * a.ntab * sizeof(TabT) : 0;
    return transpose ? launch_staged(k_jt32s<NB, TabT, U>, s, a, bytes)
                     : launch_staged(k_j32s<NB, TabT, U>, s, a, bytes);
}

template <int NB, int U>
static hipError_t launch_staged_nbu(hipStream_t s, int tabfmt, bool transpose,
                                    const ApplyArgs& a) {
    switch (tabfmt) {
        case STAB_NODE32: return launch_staged_t<float, NB, U>(s, transpose, a);
        case STAB_NODE32Z: return launch_staged_t<NodeZ, NB, U>(s, transpose, a);
        case STAB_PAIR32: return launch_staged_t<float2, NB, U>(s, transpose, a);
        case STAB_BF16: return launch_staged_t<uint32_t, NB, U>(s, transpose, a);
        // the series' own loop is long: at most four entries per step (no spills)
        case STAB_SERIES: return launch_staged_t<SinCoef, NB, (U > 4 ? 4 : U)>(s, transpose, a);
    }
    return hipErrorInvalidValue;
}

template <int NB>
static hipError_t launch_staged_nb(hipStream_t s, int tabfmt, bool transpose, const ApplyArgs& a) {
    switch (a.unroll) {
        case 1: return launch_staged_nbu<NB, 1>(s, tabfmt, transpose, a);
        case 2: return launch_staged_nbu<NB, 2>(s, tabfmt, transpose, a);
        case 4: return launch_staged_nbu<NB, 4>(s, tabfmt, transpose, a);
        case 8: return launch_staged_nbu<NB, 8>(s, tabfmt, transpose, a);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_apply_staged(hipStream_t s, int tabfmt, bool transpose, const ApplyArgs& a) {
    switch (a.nb) {
        case 1: return launch_staged_nb<1>(s, tabfmt, transpose, a);
        case 2: return launch_staged_nb<2>(s, tabfmt, transpose, a);
        case 3: return launch_staged_nb<3>(s, tabfmt, transpose, a);
        case 4: return launch_staged_nb<4>(s, tabfmt, transpose, a);
    }
    return hipErrorInvalidValue;
}

// Sensitivity coverage / diag(J^T J): the staged J^T kernel in MODE 1 / 2
// (four entries per step) with per-pair weights from k_coverage_weights.
template <int NB, int MODE>
static hipError_t launch_coverage_nb(hipStream_t s, int tabfmt, const ApplyArgs& a) {
    // no zero-topped instantiation here: the select of the plain node
    // format gives the same values on that table
    if (tabfmt == STAB_NODE32Z) tabfmt = STAB_NODE32;
    switch (tabfmt) {
        case STAB_NODE32:
            return launch_staged(k_jt32s<NB, float, 4, MODE>, s, a, (size_t)NB * a.ntab * 4);
        case STAB_PAIR32:
            return launch_staged(k_jt32s<NB, float2, 4, MODE>, s, a, (size_t)NB * a.ntab * 8);
        case STAB_BF16:
            return launch_staged(k_jt32s<NB, uint32_t, 4, MODE>, s, a, (size_t)NB * a.ntab * 4);
        case STAB_SERIES: return launch_staged(k_jt32s<NB, SinCoef, 4, MODE>, s, a, 0);
    }
    return hipErrorInvalidValue;
}

template <int MODE>
static hipError_t launch_coverage_m(hipStream_t s, int tabfmt, const ApplyArgs& a) {
    switch (a.nb) {
        case 1: return launch_coverage_nb<1, MODE>(s, tabfmt, a);
        case 2: return launch_coverage_nb<2, MODE>(s, tabfmt, a);
        case 3: return launch_coverage_nb<3, MODE>(s, tabfmt, a);
        case 4: return launch_coverage_nb<4, MODE>(s, tabfmt, a);
    }
    return hipErrorInvalidValue;
}

// Weights of the coverage passes times wscale, a power of two that keeps them
// in the normal FP32 range (C_p^2 is ~1e-42 for millimetre voxels).
__global__ void k_coverage_weights(const double* __restrict__ C, const int32_t* __restrict__ kptr,
                                   int64_t Mk, int nb, int mode, double wscale,
                                   float* __restrict__ w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Mk * (int64_t)nb) return;
    const int64_t k = i % Mk;
    const double m = (double)(kptr[k + 1] - kptr[k]);
    w[i] = (float)((mode == 1 ? fabs(C[k]) * m : C[k] * C[k] * m) * wscale);
}

hipError_t launch_coverage(hipStream_t s, int tabfmt, int mode, const ApplyArgs& a,
                           const double* C, const int32_t* kptr, double wscale, float* w) {
    const int64_t n = a.M * (int64_t)a.nb;
    if (n > 0)
        hipLaunchKernelGGL(k_coverage_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           C, kptr, a.M, a.nb, mode, wscale, w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ApplyArgs b = a;
    b.w = w;
    return mode == 1 ? launch_coverage_m<1>(s, tabfmt, b) : launch_coverage_m<2>(s, tabfmt, b);
}

// ------------------------------------------------------------ J reduction
//
// Pairs are grouped by 64 consecutive (internal) indices.  A tile's entry
// list is sorted by pair, so a group's entries in one tile form a single
// contiguous run; the pre-pass records, per group and in tile order, a
// descriptor (first entry of the run, 64-bit mask of the group's pairs
// present).  Lane i of the group's workgroup owns pair 64 g + i and reads its
// partial at run start + popcount(mask below bit i): coalesced reads, FP64
// sums in tile order, wavefronts combined in a fixed order.

struct RunDesc {
    int64_t start;
    uint64_t mask;
};

__global__ void k_group_count(const int64_t* __restrict__ tptr, const Entry* __restrict__ ents,
                              int64_t n_act, int64_t chunk, int64_t G, int32_t* __restrict__ cnt) {
    const int64_t c = blockIdx.x;
    const int64_t a0 = c * chunk;
    const int64_t a1 = min(n_act, a0 + chunk);
    int32_t* row = cnt + c * G;
    for (int64_t a = a0; a < a1; ++a) {
        const int64_t e0 = tptr[a], e1 = tptr[a + 1];
        for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
            const int g = ents[e].p >> 6;
            if (e == e0 || (ents[e - 1].p >> 6) != g) atomicAdd(&row[g], 1);
        }
    }
}

__global__ void k_group_fill(const int64_t* __restrict__ tptr, const Entry* __restrict__ ents,
                             int64_t n_act, int64_t chunk, int64_t G, int32_t* __restrict__ cnt,
                             const int64_t* __restrict__ gptr, RunDesc* __restrict__ desc) {
    const int64_t c = blockIdx.x;
    const int64_t a0 = c * chunk;
    const int64_t a1 = min(n_act, a0 + chunk);
    int32_t* row = cnt + c * G;
    for (int64_t a = a0; a < a1; ++a) {
        const int64_t e0 = tptr[a], e1 = tptr[a + 1];
        for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
            const int g = ents[e].p >> 6;
            if (e != e0 && (ents[e - 1].p >> 6) == g) continue;
            uint64_t mask = 0;
            for (int64_t k = e; k < e1 && (ents[k].p >> 6) == g; ++k)
                mask |= 1ull << (ents[k].p & 63);
            const int32_t slot = atomicAdd(&row[g], 1);
            RunDesc d;
            d.start = e;
            d.mask = mask;
            desc[gptr[g] + slot] = d;
        }
        __syncthreads();
    }
}

hipError_t launch_group_count(hipStream_t s, const int64_t* tptr, const Entry* ents,
                              int64_t n_act, int64_t chunk, int64_t G, int32_t* cnt) {
    const int64_t nc = (n_act + chunk - 1) / chunk;
    if (nc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_group_count, dim3((unsigned)nc), dim3(256), 0, s, tptr, ents, n_act,
                       chunk, G, cnt);
    return hipGetLastError();
}

hipError_t launch_group_fill(hipStream_t s, const int64_t* tptr, const Entry* ents,
                             int64_t n_act, int64_t chunk, int64_t G, int32_t* cnt,
                             const int64_t* gptr, void* desc) {
    const int64_t nc = (n_act + chunk - 1) / chunk;
    if (nc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_group_fill, dim3((unsigned)nc), dim3(256), 0, s, tptr, ents, n_act,
                       chunk, G, cnt, gptr, static_cast<RunDesc*>(desc));
    return hipGetLastError();
}

// ------------------------------------------------ source-grouped entry lists
//
// One workgroup per tile.  deg[q]: entries of the tile with endpoint q;
// each entry's source is its endpoint of larger degree (ties: the lower
// index), cnt[q] the entries with source q; gcnt[q] of them (whole fours)
// go to the grouped part, the rest to the other part.  Ranks within a source
// follow the pair order (deterministic).  Steps of eight: the grouped part's
// and the rest's are interleaved evenly (Bresenham) when the step map fits
// in LDS, else the grouped steps come first.

// Source | receiver word of the staged copies (transducers below kCopyMaxTx).
__device__ __forceinline__ uint32_t copy_sr(uint32_t s, uint32_t r, uint32_t bands) {
    return s | (r << 14) | (bands << 28);
}

constexpr int kGroupThreads = 256;
constexpr int kGroupMaxSteps = 4096;

__device__ __forceinline__ int group_source(const int* deg, uint32_t sr) {
    const int s = (int)(sr & 0xffffu), r = (int)(sr >> 16);
    return (deg[s] > deg[r] || (deg[s] == deg[r] && s <= r)) ? s : r;
}

__global__ __launch_bounds__(kGroupThreads) void k_group_order(
    const int64_t* __restrict__ tptr, const Entry* __restrict__ ents,
    const uint8_t* __restrict__ bmask, int n_tx, const int64_t* __restrict__ gtptr,
    Entry3* __restrict__ gents) {
    __shared__ int deg[kGroupMaxTx], cnt[kGroupMaxTx], gcnt[kGroupMaxTx];
    __shared__ int gstart[kGroupMaxTx], rstart[kGroupMaxTx], run[kGroupMaxTx];
    __shared__ int smap[kGroupMaxSteps];
    __shared__ int s_src[kGroupThreads];
    __shared__ int s_n[3];   // grouped entries, grouped steps, 1 if smap is used
    const int64_t a = blockIdx.x;
    const int64_t t0 = tptr[a];
    const int n = (int)(tptr[a + 1] - t0);
    const int64_t o0 = gtptr[a];
    const int nout = (int)(gtptr[a + 1] - o0);
    const int tid = (int)threadIdx.x;
    for (int q = tid; q < n_tx; q += kGroupThreads) {
        deg[q] = 0;
        cnt[q] = 0;
        run[q] = 0;
    }
    __syncthreads();
    for (int e = tid; e < n; e += kGroupThreads) {
        const uint32_t sr = ents[t0 + e].sr;
        atomicAdd(&deg[sr & 0xffffu], 1);
        atomicAdd(&deg[sr >> 16], 1);
    }
    __syncthreads();
    for (int e = tid; e < n; e += kGroupThreads)
        atomicAdd(&cnt[group_source(deg, ents[t0 + e].sr)], 1);
    __syncthreads();
    if (tid == 0) {
        int P = 0, last = -1;
        for (int q = 0; q < n_tx; ++q) {
            if (cnt[q] >= 4) last = q;
            P += cnt[q] & ~3;
        }
        // an odd number of grouped fours: the last one joins the rest
        const int drop = (P & 4) ? last : -1;
        int gp = 0, rp = 0;
        for (int q = 0; q < n_tx; ++q) {
            const int gq = (cnt[q] & ~3) - (q == drop ? 4 : 0);
            gcnt[q] = gq;
            gstart[q] = gp;
            rstart[q] = rp;
            gp += gq;
            rp += cnt[q] - gq;
        }
        const int H = nout / 8, Hg = gp / 8, Hr = H - Hg;
        s_n[0] = gp;
        s_n[1] = Hg;
        s_n[2] = H <= kGroupMaxSteps;
        if (H <= kGroupMaxSteps) {
            int kg = 0, kr = 0;
            for (int i = 0; i < H; ++i) {
                const bool rest = (int64_t)(i + 1) * Hr / H > (int64_t)i * Hr / H;
                if (rest)
                    smap[Hg + kr++] = i;
                else
                    smap[kg++] = i;
            }
        }
    }
    __syncthreads();
    const int P = s_n[0], Hg = s_n[1];
    const bool mapped = s_n[2] != 0;
    // output position of grouped (rest = false) or rest position i
    auto place = [&](bool rest, int i) {
        const int st = (rest ? Hg : 0) + (i >> 3);
        return (mapped ? smap[st] : st) * 8 + (i & 7);
    };
    for (int base = 0; base < n; base += kGroupThreads) {
        const int e = base + tid;
        int q = -1;
        Entry E;
        if (e < n) {
            E = ents[t0 + e];
            q = group_source(deg, E.sr);
        }
        s_src[tid] = q;
        __syncthreads();
        int rank = 0;
        if (q >= 0) {
            for (int k = 0; k < tid; ++k) rank += s_src[k] == q;
            rank += run[q];
        }
        __syncthreads();
        if (q >= 0) {
            atomicAdd(&run[q], 1);
            const bool rest = rank >= gcnt[q];
            const int pos = place(rest, rest ? rstart[q] + rank - gcnt[q] : gstart[q] + rank);
            const int s = (int)(E.sr & 0xffffu), r = (int)(E.sr >> 16);
            Entry3 O;
            O.p = E.p;
            O.sr = copy_sr((uint32_t)q, (uint32_t)(q == s ? r : s), bmask[t0 + e]);
            O.R0hi = E.R0hi;
            gents[o0 + pos] = O;
        }
        __syncthreads();
    }
    // padding: zero kernel value (the detour is far beyond any table, no band
    // flagged), pair 0, transducer 0 at both ends
    const int X = n - P;
    if (tid < nout - n) {
        Entry3 O;
        O.p = 0;
        O.sr = 0;
        O.R0hi = 3.0e38f;
        gents[o0 + place(true, X + tid)] = O;
    }
}

__global__ void k_pack_txc32(const TxConst* __restrict__ in, int64_t n,
                             TxConst32* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const TxConst c = in[i];
        TxConst32 o;
        o.d2x = (float)c.d2x;
        o.d2y = (float)c.d2y;
        o.d2z = (float)c.d2z;
        o.cq = (float)c.cq;
        o.D0f = c.D0f;
        o.Q0f = c.Q0f;
        out[i] = o;
    }
}

hipError_t launch_pack_txc32(hipStream_t s, const TxConst* txc, int64_t n, TxConst32* out) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_txc32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, txc, n,
                       out);
    return hipGetLastError();
}

__global__ void k_pack_j_entries(const Entry* __restrict__ in, const uint8_t* __restrict__ bm,
                                 int64_t n, uint2* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = make_uint2(copy_sr(in[i].sr & 0xffffu, in[i].sr >> 16, bm[i]),
                            __float_as_uint(in[i].R0hi));
}

hipError_t launch_pack_j_entries(hipStream_t s, const Entry* ents, const uint8_t* bmask,
                                 int64_t n, uint32_t* out) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_j_entries, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ents,
                       bmask, n, reinterpret_cast<uint2*>(out));
    return hipGetLastError();
}

// One workgroup per tile: the culling bound of each entry (as in k_cull)
// against every band's cut radius.
struct BandCuts {
    double r[kMaxBands];
};

__global__ __launch_bounds__(256) void k_band_masks(const TxConst* __restrict__ txc,
                                                    int64_t n_tx, const double* __restrict__ L,
                                                    double hwx, double hwy, double hwz,
                                                    BandCuts cut, int nb,
                                                    const int64_t* __restrict__ tptr,
                                                    const Entry* __restrict__ ents,
                                                    uint8_t* __restrict__ bmask) {
    const int64_t a = blockIdx.x;
    const TxConst* row = txc + a * n_tx;
    for (int64_t e = tptr[a] + threadIdx.x; e < tptr[a + 1]; e += blockDim.x) {
        const Entry E = ents[e];
        const TxConst A = row[E.sr & 0xffffu], B = row[E.sr >> 16];
        const double R0 = (double)A.D0f + (double)B.D0f - L[E.p];
        const double ia = 0.5 / (double)A.D0f, ib = 0.5 / (double)B.D0f;
        const double gx = A.d2x * ia + B.d2x * ib;
        const double gy = A.d2y * ia + B.d2y * ib;
        const double gz = A.d2z * ia + B.d2z * ib;
        const double lb = R0 - (fabs(gx) * hwx + fabs(gy) * hwy + fabs(gz) * hwz);
        uint32_t m = 0;
        for (int b = 0; b < nb; ++b) m |= (lb < cut.r[b] ? 1u : 0u) << b;
        bmask[e] = (uint8_t)m;
    }
}

hipError_t launch_band_masks(hipStream_t s, const int32_t* tiles, int64_t n_act,
                             const TxConst* txc, int64_t n_tx, const double* L,
                             const GridGeom& g, const double* r_cut, int nb,
                             const int64_t* tptr, const Entry* ents, uint8_t* bmask) {
    (void)tiles;
    if (n_act == 0) return hipSuccess;
    if (nb < 1 || nb > kMaxBands) return hipErrorInvalidValue;
    BandCuts cut{};
    for (int b = 0; b < nb; ++b) cut.r[b] = r_cut[b];
    const double hwx = 0.5 * (kTile - 1) * g.spacing[0];
    const double hwy = 0.5 * (kTile - 1) * g.spacing[1];
    const double hwz = 0.5 * (kTile - 1) * g.spacing[2];
    hipLaunchKernelGGL(k_band_masks, dim3((unsigned)n_act), dim3(256), 0, s, txc, n_tx, L, hwx,
                       hwy, hwz, cut, nb, tptr, ents, bmask);
    return hipGetLastError();
}

__global__ void k_pack_jt_entries(const Entry* __restrict__ in, const uint8_t* __restrict__ bm,
                                  int64_t n, Entry3* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        Entry3 o;
        o.p = in[i].p;
        o.sr = copy_sr(in[i].sr & 0xffffu, in[i].sr >> 16, bm[i]);
        o.R0hi = in[i].R0hi;
        out[i] = o;
    }
}

hipError_t launch_pack_jt_entries(hipStream_t s, const Entry* ents, const uint8_t* bmask,
                                  int64_t n, Entry3* out) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_jt_entries, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       ents, bmask, n, out);
    return hipGetLastError();
}

hipError_t launch_group_order(hipStream_t s, const int64_t* tptr, const Entry* ents,
                              const uint8_t* bmask, int64_t n_act, int n_tx,
                              const int64_t* gtptr, Entry3* gents) {
    if (n_act == 0) return hipSuccess;
    if (n_tx > kGroupMaxTx) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_group_order, dim3((unsigned)n_act), dim3(kGroupThreads), 0, s, tptr,
                       ents, bmask, n_tx, gtptr, gents);
    return hipGetLastError();
}

constexpr int kReduceWaves = 8;

// Each 64-pair group is split into S slices of its descriptor list (one
// workgroup each, so that small pair counts still fill the device); a slice
// writes its FP64 sums to red[b][slice][p], and k_reduce_final adds the S
// slices in order.
template <class T>
__global__ __launch_bounds__(64 * kReduceWaves) void k_reduce(
    const T* __restrict__ part, int64_t nnz, const int64_t* __restrict__ gptr,
    const RunDesc* __restrict__ desc, int64_t Mk, int nb, int S, double* __restrict__ red) {
    __shared__ double s_acc[kReduceWaves][64];
    const int64_t g = blockIdx.x;
    const int sl = (int)blockIdx.y;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t d0 = gptr[g], len = gptr[g + 1] - d0;
    const int64_t s0 = d0 + len * sl / S, s1 = d0 + len * (sl + 1) / S;
    const int64_t chunk = (s1 - s0 + kReduceWaves - 1) / kReduceWaves;
    const int64_t k0 = min(s1, s0 + wave * chunk), k1 = min(s1, k0 + chunk);
    const int64_t p = 64 * g + lane;
    for (int b = 0; b < nb; ++b) {
        const T* __restrict__ pb = part + (int64_t)b * nnz;
        double acc = 0.0;
        int64_t k = k0;
        // 8 descriptors per step: their gathers are issued together (the
        // index is always valid, absent pairs add zero), summed in order.
        // The next step's descriptors are requested once this step's gathers
        // are in flight, so the two latencies overlap.
        RunDesc dn[8];
        if (k + 8 <= k1) {
#pragma unroll
            for (int u = 0; u < 8; ++u) dn[u] = desc[k + u];
        }
        for (; k + 8 <= k1; k += 8) {
            RunDesc d[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) d[u] = dn[u];
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool on = (d[u].mask >> lane) & 1ull;
                v[u] = pb[d[u].start + (on ? __popcll(d[u].mask & below) : 0)];
            }
            if (k + 16 <= k1) {
#pragma unroll
                for (int u = 0; u < 8; ++u) dn[u] = desc[k + 8 + u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool on = (d[u].mask >> lane) & 1ull;
                acc += on ? (double)v[u] : 0.0;
            }
        }
        for (; k < k1; ++k) {
            const RunDesc d = desc[k];
            if ((d.mask >> lane) & 1ull) acc += (double)pb[d.start + __popcll(d.mask & below)];
        }
        s_acc[wave][lane] = acc;
        __syncthreads();
        if (wave == 0 && p < Mk) {
            double t = s_acc[0][lane];
            for (int w = 1; w < kReduceWaves; ++w) t += s_acc[w][lane];
            red[((int64_t)b * S + sl) * Mk + p] = t;
        }
        __syncthreads();
    }
}

// dT[b][i] = C_p * sum of the slices, for every caller pair i of group p.
template <class T>
__global__ void k_reduce_final(const double* __restrict__ red, int64_t Mk, int64_t M, int nb,
                               int S, const double* __restrict__ C,
                               const int32_t* __restrict__ kptr,
                               const int32_t* __restrict__ kidx, T* __restrict__ dT) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Mk * nb) return;
    const int64_t b = i / Mk, p = i - b * Mk;
    double t = 0.0;
    for (int sl = 0; sl < S; ++sl) t += red[(b * S + sl) * Mk + p];
    const T y = (T)(C[p] * t);
    for (int32_t j = kptr[p]; j < kptr[p + 1]; ++j) dT[b * M + kidx[j]] = y;
}

// As many (group, slice) workgroups as are resident at once on the device
// (four 512-thread workgroups per CU), rounded down so that they all start
// in one wave of dispatch: a second, partly filled wave would cost almost a
// whole latency-bound pass.
int reduce_slices(int64_t Mk, int n_cu) {
    const int64_t G = (Mk + 63) / 64;
    const int64_t want = 4 * (int64_t)std::max(n_cu, 1) / std::max<int64_t>(G, 1);
    return (int)std::min<int64_t>(std::max<int64_t>(want, 1), 64);
}

hipError_t launch_reduce(hipStream_t s, bool fp64, const void* part, int64_t nnz,
                         const int64_t* gptr, const void* desc, const double* C,
                         const int32_t* kptr, const int32_t* kidx, int64_t Mk, int64_t M, int nb,
                         int S, double* red, void* dT) {
    const int64_t G = (Mk + 63) / 64;
    if (G == 0) return hipSuccess;
    const RunDesc* d = static_cast<const RunDesc*>(desc);
    const unsigned nf = (unsigned)((Mk * nb + 255) / 256);
    if (fp64) {
        hipLaunchKernelGGL(k_reduce<double>, dim3((unsigned)G, (unsigned)S),
                           dim3(64 * kReduceWaves), 0, s, (const double*)part, nnz, gptr, d, Mk,
                           nb, S, red);
        hipLaunchKernelGGL(k_reduce_final<double>, dim3(nf), dim3(256), 0, s, red, Mk, M, nb, S,
                           C, kptr, kidx, (double*)dT);
    } else {
        hipLaunchKernelGGL(k_reduce<float>, dim3((unsigned)G, (unsigned)S),
                           dim3(64 * kReduceWaves), 0, s, (const float*)part, nnz, gptr, d, Mk,
                           nb, S, red);
        hipLaunchKernelGGL(k_reduce_final<float>, dim3(nf), dim3(256), 0, s, red, Mk, M, nb, S,
                           C, kptr, kidx, (float*)dT);
    }
    return hipGetLastError();
}


// ----------------------------------------------- batched point-spread functions
//
// PSF_k = J^T J e_{v_k} / sigma^2 for a batch of voxels v_k (eq. resolution_2).
//
// Step 1 (k_psf_cols): the J^T weights of the data J e_{v_k} / sigma^2,
//   W[b][p][k] = C_p^2 h_b(R_{p, v_k}) / (R_xs R_xr sigma^2),
// are non-zero only for the entries of v_k's tile: one wavefront per voxel,
// lanes over those entries.
//
// Step 2 (k_psf32): per tile, PSF[k][j] = sum_e H[j][e] W[e][k] with
// H[j][e] = h(R) / (R_xs R_xr) for voxel j of the tile and entry e: a dense
// (64 x E) (E x n) product, done on the matrix cores with
// v_mfma_f32_32x32x2f32 (FP32 operands and accumulation).  Each wavefront
// owns 32 right-hand sides (the N dimension) and walks all entries of the
// tile two at a time (K = 2), so there is no cross-wave reduction; the 64
// voxels are two M = 32 blocks.  H comes from the LDS-staged distances as in
// the single-RHS kernels.

using f32x16 = __attribute__((__vector_size__(16 * sizeof(float)))) float;

// The PSF kernels' output step: one [32][33] float LDS slot per wave (up to
// 16 waves), taken from the start of the dynamic LDS once the tile is done.
constexpr int kPsfOutSlot = 32 * 33;
constexpr size_t kPsfOutLds = 16 * kPsfOutSlot * sizeof(float);

// Writes a wave's 64-voxel x 32-column block of PSFs (columns k0 .. k0 + 31
// below n) of active tile a.  The block is two 32 x 32 matrix-core results, lo for
// voxels 0-31 and hi for 32-63, where register q of lane l holds voxel
// 8 (q / 4) + 4 (l / 32) + q % 4 of the half in column l % 32.  Each half
// goes through the wave's LDS slot so that a store covers 32 voxels of two
// columns (runs of four x-neighbours) rather than one voxel in each of 32
// columns a whole volume apart; with an x extent that is a multiple of four
// a lane stores a row of four x-neighbours as one float4.  Every lane of the
// wave takes part; the workgroup must be done with the LDS.
template <class V>
__device__ __forceinline__ void store_psf_block(const ApplyArgs& A, int64_t a, const V& c_lo,
                                                const V& c_hi, int k0, int n, int wave,
                                                int lane, float* __restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    float* slot = reinterpret_cast<float*>(smem) + wave * kPsfOutSlot;
    const int64_t N = (int64_t)A.g.dims[0] * A.g.dims[1] * A.g.dims[2];
    const int col = lane & 31, up = lane >> 5;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int q = 0; q < 16; ++q)
            slot[col * 33 + 8 * (q / 4) + 4 * up + (q & 3)] = h ? c_hi[q] : c_lo[q];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (A.g.dims[0] % 4 == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
            // rows of four x-neighbours stay inside the grid and 16-byte
            // aligned (x extent a multiple of four, 16-byte aligned output):
            // lane = (row r of the half, column c % 8), one float4 store per
            // row and column
            const int r = lane & 7, cq = lane >> 3;
            bool inside, act;
            int64_t vidx, v[3];
            voxel_of_lane(A, a, 4 * r + 32 * h, inside, act, vidx, v);
            const uint32_t m = inside ? *reinterpret_cast<const uint32_t*>(A.mask + vidx) : 0u;
#pragma unroll
            for (int it = 0; it < 4; ++it) {
                const int c = 8 * it + cq;
                const float* sv = slot + c * 33 + 4 * r;
                float4 q;
                q.x = (m & 0xffu) ? sv[0] : 0.0f;
                q.y = (m & 0xff00u) ? sv[1] : 0.0f;
                q.z = (m & 0xff0000u) ? sv[2] : 0.0f;
                q.w = (m & 0xff000000u) ? sv[3] : 0.0f;
                if (inside && k0 + c < n)
                    *reinterpret_cast<float4*>(out + (int64_t)(k0 + c) * N + vidx) = q;
            }
        } else {
            bool inside, act;
            int64_t vidx, v[3];
            voxel_of_lane(A, a, col + 32 * h, inside, act, vidx, v);
#pragma unroll
            for (int it = 0; it < 16; ++it) {
                const int c = 2 * it + up;
                const float val = slot[c * 33 + col];
                if (inside && k0 + c < n) out[(int64_t)(k0 + c) * N + vidx] = act ? val : 0.0f;
            }
        }
        // the slot's reads complete before the next half overwrites it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

// bf16(a) | bf16(b) << 16, both rounded to nearest even in one conversion.
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
    const f32x2v v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2v));
}

// Splits a pair of floats x ~ hi + lo (hi = bf16(x), lo = bf16(x - hi)) into
// packed words: hi and lo of a in the low halves, of b in the high halves.
__device__ __forceinline__ void split_bf16x2(float a, float b, uint32_t& hi, uint32_t& lo) {
    hi = pack_bf16x2(a, b);
    lo = pack_bf16x2(a - __uint_as_float(hi << 16), b - __uint_as_float(hi & 0xffff0000u));
}

// The same split of one float as one word: hi in the low half, lo in the high
// half (what split_bf16x2 gives for the float in either position).
__device__ __forceinline__ uint32_t split_word(float x) {
    const uint32_t hi = pack_bf16x2(x, 0.0f) & 0xffffu;
    return hi | (pack_bf16x2(x - __uint_as_float(hi << 16), 0.0f) << 16);
}

template <int NB, class TabT>
__global__ __launch_bounds__(64) void k_psf_cols(ApplyArgs A, const int32_t* __restrict__ ptile,
                                                 const int32_t* __restrict__ plane,
                                                 const double* __restrict__ C,
                                                 const int32_t* __restrict__ kptr, double s2,
                                                 float* __restrict__ W, int64_t ldw, bool packed) {
    const int k = blockIdx.x;
    const int64_t a = ptile[k];
    const int l = plane[k];
    const double ux = ((double)(l & 3) - 1.5) * A.g.spacing[0];
    const double uy = ((double)((l >> 2) & 3) - 1.5) * A.g.spacing[1];
    const double uz = ((double)(l >> 4) - 1.5) * A.g.spacing[2];
    const double uu = ux * ux + uy * uy + uz * uz;
    const TxConst* __restrict__ row = A.txc + a * A.n_tx;
    const TabT* tab = static_cast<const TabT*>(A.tab);
    const float nm1 = (float)(A.ntab - 1);
    for (int64_t e = A.tptr[a] + threadIdx.x; e < A.tptr[a + 1]; e += 64) {
        const Entry E = A.ents[e];
        const int s = (int)(E.sr & 0xffffu), r = (int)(E.sr >> 16);
        float ds, gs, dr, gr;
        dist32(row[s], ux, uy, uz, uu, ds, gs);
        dist32(row[r], ux, uy, uz, uu, dr, gr);
        const float R = (ds + dr) + E.R0hi;
        // a kernel pair stands for kptr[p+1] - kptr[p] identical rows of J
        const double c = C[E.p];
        const double m = (double)(kptr[E.p + 1] - kptr[E.p]);
        const float f = (float)(c * c * m * s2) * (gs * gr);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const float v = lookup(tab + b * A.ntab, R, A.inv_dr[b], nm1) * f;
            const int64_t o = ((int64_t)b * A.M + E.p) * ldw + k;
            if (packed)
                reinterpret_cast<uint32_t*>(W)[o] = split_word(v);
            else
                W[o] = v;
        }
    }
}

// H of one entry and band for every lane (voxel) of the tile.
template <class TabT>
__device__ __forceinline__ float psf_h(const ApplyArgs& A, const TabT* st, const float2* sx,
                                       const Entry& E, int b, float nm1, int lane) {
    const int s = (int)(E.sr & 0xffffu), r = (int)(E.sr >> 16);
    const float2 vs = sx[s * 64 + lane], vr = sx[r * 64 + lane];
    const float x0 = fmaf(E.R0hi, A.inv_dr[0], vs.x + vr.x);
    const float xb = b == 0 ? x0 : x0 * A.xr[b];
    return lookup_x(st + b * A.ntab, table_x(xb, nm1), nm1) * (vs.y * vr.y);
}

// Entries per chunk of the PSF contraction (H of a chunk is shared in LDS).
template <int NB>
constexpr int psf_chunk() { return NB == 1 ? 64 : (NB == 2 ? 32 : (NB == 3 ? 16 : 8)); }

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Runs of kXcdRun consecutive tiles, which share most of their
// pairs, go to one XCD (one L2); the runs are dealt out round-robin so that
// every XCD sees every part of the volume (entry counts vary strongly with
// the distance from the transducers).  The grid is padded to whole rounds;
// blocks past the last tile return at once.
constexpr int kXcds = 8;
constexpr int kXcdRun = 128;

__device__ __forceinline__ int64_t xcd_tile(int64_t b) {
    const int64_t x = b % kXcds, i = b / kXcds;
    return (i / kXcdRun) * (kXcds * kXcdRun) + x * kXcdRun + i % kXcdRun;
}

inline int64_t xcd_grid(int64_t n) {
    const int64_t round = (int64_t)kXcds * kXcdRun;
    return (n + round - 1) / round * round;
}

// Weights of the PSF contractions, W [nb][M][ldw] FP32 (split words for the
// split-BF16 contraction, read through the same path): wrow is a wave's
// block of columns in one band (uniform), the gather for kernel pair p and
// the lane's column one 24-bit multiply-add on a 32-bit byte offset (the
// launches require M ldw < 2^30 and ldw < 2^22).  The chunk producers give
// padding entries pair 0: their H is exactly zero and W is finite, so the
// row they read adds nothing.
__device__ __forceinline__ float psf_weight(const float* wrow, int p, uint32_t ldw4,
                                            uint32_t col4) {
    const uint32_t off = __umul24((uint32_t)p, ldw4) + col4;
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(wrow) + off);
}

// Entries a wave of a chunk producer evaluates together: their loads are
// issued at once, so the entry -> distance -> table chains overlap.
constexpr int kProduceBatch = 4;

// The batch of entries c0 + i0 + u * W_ (u < kProduceBatch) of a chunk of CH:
// slots past the chunk or the tile take entry t0 (always valid) and ok = 0.
template <int CH>
__device__ __forceinline__ void produce_batch(const ApplyArgs& A, int64_t c0, int i0, int W_,
                                              int64_t t0, int64_t t1,
                                              Entry (&E)[kProduceBatch],
                                              bool (&ok)[kProduceBatch]) {
#pragma unroll
    for (int u = 0; u < kProduceBatch; ++u) {
        const int i = i0 + u * W_;
        const int64_t e = c0 + i;
        ok[u] = i < CH && e < t1;
        E[u] = A.ents[ok[u] ? e : t0];
    }
}

// H (and the pair index) of chunk entries c0 .. c0 + CH - 1 into one buffer;
// the workgroup's waves split the entries.
template <int NB, int CH, class TabT>
__device__ __forceinline__ void psf_chunk_h(const ApplyArgs& A, const TabT* st, const float2* sx,
                                            float* hb, int* pb, int64_t c0, int64_t t0,
                                            int64_t t1, float nm1, int wave, int W_, int lane) {
    for (int i0 = wave; i0 < CH; i0 += kProduceBatch * W_) {
        Entry E[kProduceBatch];
        bool ok[kProduceBatch];
        produce_batch<CH>(A, c0, i0, W_, t0, t1, E, ok);
#pragma unroll
        for (int u = 0; u < kProduceBatch; ++u) {
            const int i = i0 + u * W_;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const float h = psf_h(A, st, sx, E[u], b, nm1, lane);
                if (i < CH) hb[(b * CH + i) * 64 + lane] = ok[u] ? h : 0.0f;
            }
            if (lane == 0 && i < CH) pb[i] = ok[u] ? E[u].p : 0;
        }
    }
}

template <int NB, class TabT>
__global__ __launch_bounds__(1024) void k_psf32(ApplyArgs A, const float* __restrict__ W,
                                                int64_t ldw, int n, float* __restrict__ out) {
    constexpr int CH = psf_chunk<NB>();
    constexpr int HB = NB * CH * 64;   // floats of one H buffer
    const TabT* st = stage_table<TabT>(A, NB);
    float2* sx = staged_tx<TabT>(A, NB);
    // after the staged distances: two H buffers [NB][CH][64] and two index
    // buffers [CH] (chunk c in buffer c % 2)
    float* hbuf = reinterpret_cast<float*>(sx + A.n_tx * 64);
    int* pbuf = reinterpret_cast<int*>(hbuf + 2 * HB);
    const int64_t a = xcd_tile(blockIdx.x);
    if (a >= A.n_act) return;
    const int lane = threadIdx.x & 63;
    const LaneVox V = lane_vox(A, a, lane);
    stage_distances(A, a, V, sx, lane, 0, (int)A.n_tx);   // one block: all transducers
    const int W_ = (int)(blockDim.x >> 6);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int k0 = ((int)blockIdx.y * W_ + wave) * 32;
    const bool active = k0 < n;   // wave-uniform; idle waves still help with H
    const float nm1 = (float)(A.ntab - 1);
    const int64_t t0 = A.tptr[a], t1 = A.tptr[a + 1];
    const int col = lane & 31;
    const int up = lane >> 5;
    const uint32_t ldw4 = 4u * (uint32_t)ldw, col4 = 4u * (uint32_t)col;
    f32x16 c_lo = {}, c_hi = {};
    if (t0 < t1)
        psf_chunk_h<NB, CH>(A, st, sx, hbuf, pbuf, t0, t0, t1, nm1, wave, W_, lane);
    __syncthreads();
    int buf = 0;
    for (int64_t c0 = t0; c0 < t1; c0 += CH, buf ^= 1) {
        const float* hb = hbuf + buf * HB;
        const int* pb = pbuf + buf * CH;
        // this chunk's weights (requested first), the next chunk's H (into
        // the other buffer), then this chunk's matrix-core steps
        float bw[NB][CH / 2];
        if (active) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int j = 0; j < CH / 2; ++j)
                    bw[b][j] = psf_weight(W + ((int64_t)b * A.M) * ldw + k0, pb[2 * j + up],
                                          ldw4, col4);
        }
        if (c0 + CH < t1)
            psf_chunk_h<NB, CH>(A, st, sx, hbuf + (buf ^ 1) * HB, pbuf + (buf ^ 1) * CH, c0 + CH,
                                t0, t1, nm1, wave, W_, lane);
        if (active) {
            // A of voxels 0-31: lanes 0-31 entry 2j, lanes 32-63 entry 2j+1;
            // voxels 32-63 likewise, 32 floats further on.  The operands of
            // the next group of K-steps are read while the current group's
            // matrix-core steps run.
            constexpr int KS = CH / 2, G = KS < 8 ? KS : 8;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const float* hb0 = hb + b * CH * 64 + up * 64 + col;
                float al[G], ah[G];
#pragma unroll
                for (int jj = 0; jj < G; ++jj) {
                    al[jj] = hb0[2 * jj * 64];
                    ah[jj] = hb0[2 * jj * 64 + 32];
                }
#pragma unroll
                for (int g = 0; g < KS / G; ++g) {
                    float nl[G], nh[G];
                    if (g + 1 < KS / G) {
#pragma unroll
                        for (int jj = 0; jj < G; ++jj) {
                            nl[jj] = hb0[2 * ((g + 1) * G + jj) * 64];
                            nh[jj] = hb0[2 * ((g + 1) * G + jj) * 64 + 32];
                        }
                    }
                    // keep the reads above and the matrix-core steps below in
                    // this order (the scheduler would otherwise sink each read
                    // to its use and expose its latency)
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int jj = 0; jj < G; ++jj) {
                        c_lo = __builtin_amdgcn_mfma_f32_32x32x2f32(al[jj], bw[b][g * G + jj],
                                                                    c_lo, 0, 0, 0);
                        c_hi = __builtin_amdgcn_mfma_f32_32x32x2f32(ah[jj], bw[b][g * G + jj],
                                                                    c_hi, 0, 0, 0);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    if (g + 1 < KS / G) {
#pragma unroll
                        for (int jj = 0; jj < G; ++jj) {
                            al[jj] = nl[jj];
                            ah[jj] = nh[jj];
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (!active) return;
    store_psf_block(A, a, c_lo, c_hi, k0, n, wave, lane, out);
}

// ---- the same contraction with BF16 matrix-core steps, split three ways
//
// Every FP32 operand x is split as x ~ hi + lo, hi = bf16(x), lo = bf16(x -
// hi) (relative error ~2^-17), and each product is taken as hi*hi + hi*lo +
// lo*hi (the dropped lo*lo is ~2^-16 relative) on v_mfma_f32_32x32x16_bf16
// with FP32 accumulation: three BF16 steps per K = 16 block instead of eight
// FP32 K = 2 steps.  Norm-wise error ~3e-6 on PSF operands.  H is split once,
// when it is produced (all wavefronts reuse it), and kept voxel-major in LDS
// as [voxel][entry] BF16 rows of CH + 8 (16-byte aligned, conflict-free
// 16-byte reads of a lane's 8 K-values); W arrives split by its producers
// (split_word: one word per value) and is regrouped in registers.  Operand
// layout (32x32x16): A[m][k] in lane m + 32 (k / 8), element k % 8; B[k][n]
// in lane n + 32 (k / 8), element k % 8.

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16v __attribute__((ext_vector_type(16)));

constexpr int psfb3_chunk(int nb) { return nb == 1 ? 64 : (nb == 2 ? 32 : 16); }

__device__ __forceinline__ uint32_t bf16_bits(__bf16 h) {
    return (uint32_t)__builtin_bit_cast(uint16_t, h);
}

// Entry pairs a wave evaluates together in one batch of a chunk (one with
// several bands, within the registers).
template <int NB>
constexpr int psfb3_pb() { return NB == 1 ? kProduceBatch / 2 : 1; }

// Index of slot u of the batch starting at pair j0 of chunk c0, and whether it
// is a real entry (slots past the chunk or the tile read entry t0 instead).
template <int CH>
__device__ __forceinline__ int64_t psfb3_slot(int64_t c0, int j0, int u, int W_, int64_t t0,
                                              int64_t t1, bool& ok) {
    const int i2 = j0 + (u / 2) * W_;
    const int64_t e = c0 + 2 * i2 + (u & 1);
    ok = i2 < CH / 2 && e < t1;
    return ok ? e : t0;
}

// H of one batch of entry pairs split into hi / lo BF16 rows; each lane
// (voxel) writes one packed dword per pair.
template <int NB, int CH, class TabT>
__device__ __forceinline__ void psfb3_batch_h(const ApplyArgs& A, const TabT* st, const float2* sx,
                                              uint32_t* hh, uint32_t* hl, int* pb,
                                              const Entry (&E)[2 * psfb3_pb<NB>()],
                                              const bool (&ok)[2 * psfb3_pb<NB>()], int j0,
                                              float nm1, int W_, int lane) {
    constexpr int RS = (CH + 8) / 2;   // row stride in dwords
    constexpr int PB = psfb3_pb<NB>();
#pragma unroll
    for (int v = 0; v < PB; ++v) {
        const int i2 = j0 + v * W_;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            float h0 = psf_h(A, st, sx, E[2 * v], b, nm1, lane);
            float h1 = psf_h(A, st, sx, E[2 * v + 1], b, nm1, lane);
            h0 = ok[2 * v] ? h0 : 0.0f;
            h1 = ok[2 * v + 1] ? h1 : 0.0f;
            uint32_t wh, wl;
            split_bf16x2(h0, h1, wh, wl);
            const int o = (b * 64 + lane) * RS + i2;
            if (i2 < CH / 2) {
                hh[o] = wh;
                hl[o] = wl;
            }
        }
        if (lane == 0 && i2 < CH / 2) {
            pb[2 * i2] = ok[2 * v] ? E[2 * v].p : 0;
            pb[2 * i2 + 1] = ok[2 * v + 1] ? E[2 * v + 1].p : 0;
        }
    }
}

// H of entries c0 .. c0 + CH - 1; waves take batches of entry pairs, their
// entries read by scalar loads.
template <int NB, int CH, class TabT>
__device__ __forceinline__ void psfb3_chunk_h(const ApplyArgs& A, const TabT* st, const float2* sx,
                                              uint32_t* hh, uint32_t* hl, int* pb, int64_t c0,
                                              int64_t t0, int64_t t1, float nm1, int wave,
                                              int W_, int lane) {
    constexpr int PB = psfb3_pb<NB>();
    for (int j0 = wave; j0 < CH / 2; j0 += PB * W_) {
        Entry E[2 * PB];
        bool ok[2 * PB];
#pragma unroll
        for (int u = 0; u < 2 * PB; ++u) E[u] = A.ents[psfb3_slot<CH>(c0, j0, u, W_, t0, t1, ok[u])];
        psfb3_batch_h<NB, CH>(A, st, sx, hh, hl, pb, E, ok, j0, nm1, W_, lane);
    }
}

// When one batch per wave covers a chunk, the wave's entries of a chunk are
// requested one chunk ahead, through the vector memory path (the byte offset
// is moved to a VGPR, so the loads are not turned into scalar loads): they
// are counted by vmcnt, in order with the weight loads, and a scalar load in
// flight would make every LDS wait in between wait for it as well.
template <int NB, int CH>
__device__ __forceinline__ void psfb3_prefetch(const ApplyArgs& A, int64_t c0, int64_t t0,
                                               int64_t t1, int wave, int W_,
                                               u32x4 (&ev)[2 * psfb3_pb<NB>()]) {
    const char* base = reinterpret_cast<const char*>(A.ents + t0);
#pragma unroll
    for (int u = 0; u < 2 * psfb3_pb<NB>(); ++u) {
        bool ok;
        const int64_t e = psfb3_slot<CH>(c0, wave, u, W_, t0, t1, ok);
        const uint32_t off = to_vgpr((uint32_t)(e - t0) * (uint32_t)sizeof(Entry));
        ev[u] = *reinterpret_cast<const u32x4*>(base + off);
    }
}

template <int NB, class TabT>
__global__ __launch_bounds__(1024) void k_psfb3(ApplyArgs A, const float* __restrict__ W,
                                                int64_t ldw, int n, float* __restrict__ out) {
    constexpr int CH = psfb3_chunk(NB);
    constexpr int RS = (CH + 8) / 2;          // dwords per voxel row
    constexpr int HB = NB * 64 * RS;          // dwords of one hi (or lo) buffer
    const TabT* st = stage_table<TabT>(A, NB);
    float2* sx = staged_tx<TabT>(A, NB);
    // after the staged distances: two buffer sets {hi, lo, index}
    uint32_t* hbuf = reinterpret_cast<uint32_t*>(sx + A.n_tx * 64);
    int* pbuf = reinterpret_cast<int*>(hbuf + 4 * HB);
    const int64_t a = xcd_tile(blockIdx.x);
    if (a >= A.n_act) return;
    const int lane = threadIdx.x & 63;
    const LaneVox V = lane_vox(A, a, lane);
    stage_distances(A, a, V, sx, lane, 0, (int)A.n_tx);   // one block: all transducers
    const int W_ = (int)(blockDim.x >> 6);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int k0 = ((int)blockIdx.y * W_ + wave) * 32;
    const bool active = k0 < n;   // wave-uniform; idle waves still help with H
    const float nm1 = (float)(A.ntab - 1);
    const int64_t t0 = A.tptr[a], t1 = A.tptr[a + 1];
    const int col = lane & 31;
    const int up = lane >> 5;
    const uint32_t ldw4 = 4u * (uint32_t)ldw, col4 = 4u * (uint32_t)col;
    f32x16v c_lo = {}, c_hi = {};
    constexpr int PB = psfb3_pb<NB>();
    // one batch per wave covers a chunk: entries requested a chunk ahead
    const bool pre = PB * W_ >= CH / 2;
    u32x4 ev[2 * PB];
    if (pre && t0 + CH < t1) psfb3_prefetch<NB, CH>(A, t0 + CH, t0, t1, wave, W_, ev);
    if (t0 < t1)
        psfb3_chunk_h<NB, CH>(A, st, sx, hbuf, hbuf + HB, pbuf, t0, t0, t1, nm1, wave, W_, lane);
    __syncthreads();
    int buf = 0;
    for (int64_t c0 = t0; c0 < t1; c0 += CH, buf ^= 1) {
        const uint32_t* hh = hbuf + buf * 2 * HB;
        const uint32_t* hl = hh + HB;
        const int* pb = pbuf + buf * CH;
        // this chunk's weights (requested first), the next chunk's H, then
        // the split and the matrix-core steps
        uint32_t wv[NB][CH / 16][8];
        if (active) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int s = 0; s < CH / 16; ++s)
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        wv[b][s][i] = __float_as_uint(
                            psf_weight(W + ((int64_t)b * A.M) * ldw + k0,
                                       pb[16 * s + 8 * up + i], ldw4, col4));
        }
        if (c0 + CH < t1) {
            uint32_t* nh = hbuf + (buf ^ 1) * 2 * HB;
            int* np = pbuf + (buf ^ 1) * CH;
            if (pre) {
                Entry E[2 * PB];
                bool ok[2 * PB];
#pragma unroll
                for (int u = 0; u < 2 * PB; ++u) {
                    psfb3_slot<CH>(c0 + CH, wave, u, W_, t0, t1, ok[u]);
                    E[u] = __builtin_bit_cast(Entry, ev[u]);
                }
                if (c0 + 2 * CH < t1) psfb3_prefetch<NB, CH>(A, c0 + 2 * CH, t0, t1, wave, W_, ev);
                psfb3_batch_h<NB, CH>(A, st, sx, nh, nh + HB, np, E, ok, wave, nm1, W_, lane);
            } else {
                psfb3_chunk_h<NB, CH>(A, st, sx, nh, nh + HB, np, c0 + CH, t0, t1, nm1, wave, W_,
                                      lane);
            }
        }
        if (active) {
            // the split weights regrouped into hi and lo operands once they
            // are needed (their loads stay in flight over the H evaluation
            // above): one byte permutation per two values
            bf16x8 wh[NB][CH / 16], wl[NB][CH / 16];
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int s = 0; s < CH / 16; ++s) {
                    u32x4 h, l;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        h[k] = __builtin_amdgcn_perm(wv[b][s][2 * k + 1], wv[b][s][2 * k],
                                                     0x05040100u);
                        l[k] = __builtin_amdgcn_perm(wv[b][s][2 * k + 1], wv[b][s][2 * k],
                                                     0x07060302u);
                    }
                    wh[b][s] = __builtin_bit_cast(bf16x8, h);
                    wl[b][s] = __builtin_bit_cast(bf16x8, l);
                }
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int s = 0; s < CH / 16; ++s) {
                    // lane: voxel col (+ 32 for the upper block), K-values
                    // 16 s + 8 up .. + 7 (4 dwords)
                    const int o = (b * 64 + col) * RS + 8 * s + 4 * up;
                    const bf16x8 al = *reinterpret_cast<const bf16x8*>(hh + o);
                    const bf16x8 ah = *reinterpret_cast<const bf16x8*>(hh + o + 32 * RS);
                    const bf16x8 bl = *reinterpret_cast<const bf16x8*>(hl + o);
                    const bf16x8 bh = *reinterpret_cast<const bf16x8*>(hl + o + 32 * RS);
                    c_lo = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, wh[b][s], c_lo, 0, 0, 0);
                    c_hi = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, wh[b][s], c_hi, 0, 0, 0);
                    c_lo = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, wl[b][s], c_lo, 0, 0, 0);
                    c_hi = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, wl[b][s], c_hi, 0, 0, 0);
                    c_lo = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bl, wh[b][s], c_lo, 0, 0, 0);
                    c_hi = __builtin_amdgcn_mfma_f32_32x32x16_bf16(bh, wh[b][s], c_hi, 0, 0, 0);
                }
        }
        __syncthreads();
    }
    if (!active) return;
    store_psf_block(A, a, c_lo, c_hi, k0, n, wave, lane, out);
}

// ---- batched J for dense right-hand sides (Gauss-Newton Hessian blocks)
//
// part[b][e][k] = sum_j H_b[j][e] Q[k][j] for the entries e of a tile and l
// right-hand sides Q ([l][ldq] model vectors): per 64-entry chunk a dense
// (64 entries x 64 voxels)(64 voxels x 32 columns) product per wavefront on
// the BF16 matrix cores with three-way split operands (as k_psfb3).  H is
// kept entry-major ([entry][voxel] BF16 rows of 72) so a lane's 8 K-values
// (voxels) are one 16-byte read; the tile's 64 x 32 block of Q is loaded
// and split once per tile.  Each chunk's K range is the whole tile, so the
// chunk's 64 x 32 result is final and stored at once.

template <int NB, class TabT>
__global__ __launch_bounds__(1024) void k_jmb3(ApplyArgs A, const float* __restrict__ Q,
                                               int64_t ldq, int l, float* __restrict__ part) {
    constexpr int CH = 64, RS = 36;           // entries per chunk, dwords per entry row
    constexpr int HB = NB * CH * RS;          // dwords of one hi (or lo) buffer
    const TabT* st = stage_table<TabT>(A, NB);
    float2* sx = staged_tx<TabT>(A, NB);
    uint32_t* hbuf = reinterpret_cast<uint32_t*>(sx + A.n_tx * 64);
    uint16_t* hb16 = reinterpret_cast<uint16_t*>(hbuf);
    int* svid = reinterpret_cast<int*>(hbuf + 4 * HB);   // [64] model index of each voxel
    const int64_t a = xcd_tile(blockIdx.x);
    if (a >= A.n_act) return;
    const int lane = threadIdx.x & 63;
    const LaneVox V = lane_vox(A, a, lane);
    stage_distances(A, a, V, sx, lane, 0, (int)A.n_tx);   // ends with a barrier
    const int W_ = (int)(blockDim.x >> 6);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (wave == 0)
        svid[lane] = V.act ? (int)(A.nxy ? V.vidx % A.nxy : V.vidx) : -1;
    const int k0 = ((int)blockIdx.y * W_ + wave) * 32;
    const bool active = k0 < l;
    const float nm1 = (float)(A.ntab - 1);
    const int64_t t0 = A.tptr[a], t1 = A.tptr[a + 1];
    const int col = lane & 31;
    const int up = lane >> 5;
    // this wave's block of 32 partial columns: rows of wb floats
    const int lp = hess_part_ld(l);
    const int wb = min(32, lp - k0);
    float* __restrict__ pblk = part + (int64_t)k0 * A.nnz;
    // H of a chunk: waves split the entries, lane = voxel, BF16 hi / lo
    auto produce_from = [&](uint16_t* hh, uint16_t* hl, int i0, const Entry (&E)[kProduceBatch],
                            const bool (&ok)[kProduceBatch]) {
#pragma unroll
        for (int u = 0; u < kProduceBatch; ++u) {
            const int i = i0 + u * W_;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                float h = psf_h(A, st, sx, E[u], b, nm1, lane);
                h = ok[u] ? h : 0.0f;
                const __bf16 hi = (__bf16)h;
                const int o = ((b * CH + i) * RS) * 2 + lane;
                if (i < CH) {
                    hh[o] = __builtin_bit_cast(uint16_t, hi);
                    hl[o] = __builtin_bit_cast(uint16_t, (__bf16)(h - (float)hi));
                }
            }
        }
    };
    auto produce = [&](uint16_t* hh, uint16_t* hl, int64_t c0) {
        for (int i0 = wave; i0 < CH; i0 += kProduceBatch * W_) {
            Entry E[kProduceBatch];
            bool ok[kProduceBatch];
            produce_batch<CH>(A, c0, i0, W_, t0, t1, E, ok);
            produce_from(hh, hl, i0, E, ok);
        }
    };
    // one batch per wave covers a chunk: the wave's entries of the next chunk
    // are requested a chunk ahead through the vector memory path (as in
    // k_psfb3)
    const bool pre = kProduceBatch * W_ >= CH;
    const char* ebase = reinterpret_cast<const char*>(A.ents + t0);
    u32x4 ev[kProduceBatch];
    auto slot = [&](int64_t c0, int u, bool& ok) -> int64_t {
        const int i = wave + u * W_;
        const int64_t e = c0 + i;
        ok = i < CH && e < t1;
        return ok ? e : t0;
    };
    auto prefetch = [&](int64_t c0) {
#pragma unroll
        for (int u = 0; u < kProduceBatch; ++u) {
            bool ok;
            const uint32_t off = to_vgpr((uint32_t)(slot(c0, u, ok) - t0) * (uint32_t)sizeof(Entry));
            ev[u] = *reinterpret_cast<const u32x4*>(ebase + off);
        }
    };
    if (pre && t0 + CH < t1) prefetch(t0 + CH);
    if (t0 < t1) produce(hb16, hb16 + 2 * HB, t0);
    __syncthreads();
    // this wave's columns of Q on the tile's voxels, split once
    bf16x8 qh[4], ql[4];
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int vid = svid[16 * s4 + 8 * up + i];
            const float q = (active && k0 + col < l && vid >= 0)
                                ? Q[(int64_t)(k0 + col) * ldq + vid] : 0.0f;
            const __bf16 x = (__bf16)q;
            qh[s4][i] = x;
            ql[s4][i] = (__bf16)(q - (float)x);
        }
    int buf = 0;
    for (int64_t c0 = t0; c0 < t1; c0 += CH, buf ^= 1) {
        const uint32_t* hh = hbuf + buf * 2 * HB;
        const uint32_t* hl = hh + HB;
        if (c0 + CH < t1) {
            uint16_t* nh = hb16 + (buf ^ 1) * 4 * HB;
            if (pre) {
                Entry E[kProduceBatch];
                bool ok[kProduceBatch];
#pragma unroll
                for (int u = 0; u < kProduceBatch; ++u) {
                    slot(c0 + CH, u, ok[u]);
                    E[u] = __builtin_bit_cast(Entry, ev[u]);
                }
                if (c0 + 2 * CH < t1) prefetch(c0 + 2 * CH);
                produce_from(nh, nh + 2 * HB, wave, E, ok);
            } else {
                produce(nh, nh + 2 * HB, c0 + CH);
            }
        }
        if (active) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                f32x16v acc[2] = {};
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) {
                        const int o = (b * CH + 32 * mb + col) * RS + 8 * s4 + 4 * up;
                        const bf16x8 ah = *reinterpret_cast<const bf16x8*>(hh + o);
                        const bf16x8 al = *reinterpret_cast<const bf16x8*>(hl + o);
                        acc[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, qh[s4], acc[mb], 0, 0, 0);
                        acc[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, ql[s4], acc[mb], 0, 0, 0);
                        acc[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, qh[s4], acc[mb], 0, 0, 0);
                    }
                // D: register q of lane -> entry row 8 (q / 4) + 4 up + q % 4
                if (col < wb) {
#pragma unroll
                    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                        for (int q = 0; q < 16; ++q) {
                            const int64_t e = c0 + 32 * mb + 8 * (q / 4) + 4 * up + (q & 3);
                            if (e < t1) pblk[(int64_t)b * lp * A.nnz + e * wb + col] = acc[mb][q];
                        }
                }
            }
        }
        __syncthreads();
    }
}

// Per-pair sums of the batched partials over the tiles (RunDesc groups as
// in k_reduce): red[b][s][p][k] over slice s of the group's descriptors,
// FP64, descriptors in order.  A workgroup takes one (group, slice) and up
// to kRedColWaves column chunks of eight, one per wave: its waves walk the
// same descriptors, so a partial row comes from HBM once and from the CU's
// caches for its other chunks.  The partials lie in blocks of 32 columns
// (rows of 32 floats, the last block hess_part_ld(l) - 32 k), so a lane's
// eight columns are two aligned 16-byte loads.
constexpr int kRedCols = 8;
constexpr int kRedColWaves = 16;
constexpr int kRedUnroll = 8;

__global__ __launch_bounds__(64 * kRedColWaves) void k_reduce_cols(
    const float* __restrict__ part, int64_t nnz, int l, const int64_t* __restrict__ gptr,
    const RunDesc* __restrict__ desc, int64_t Mk, int nb, int S, double* __restrict__ red) {
    const int64_t g = blockIdx.x;
    const int sl = (int)blockIdx.y;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int c0 = ((int)blockIdx.z * kRedColWaves + wave) * kRedCols;
    if (c0 >= l) return;
    const int lane = threadIdx.x & 63;
    const int lp = hess_part_ld(l);
    const int cb = c0 & ~31;               // first column of c0's block
    const int wb = min(32, lp - cb);       // the block's row length
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t d0 = gptr[g], len = gptr[g + 1] - d0;
    const int64_t k0 = d0 + len * sl / S, k1 = d0 + len * (sl + 1) / S;
    const int64_t p = 64 * g + lane;
    const int nc = min(kRedCols, l - c0);
    for (int b = 0; b < nb; ++b) {
        double acc[kRedCols];
#pragma unroll
        for (int c = 0; c < kRedCols; ++c) acc[c] = 0.0;
        // kRedUnroll descriptors per step, loads first: a lane outside a run
        // reads the run's first row and adds an exact 0.0, so every sum is
        // taken in descriptor order as with one descriptor at a time
        const float* pb = part + ((int64_t)b * lp + cb) * nnz + (c0 - cb);
        auto add = [&](bool on, float4 u, float4 v) {
            acc[0] += on ? (double)u.x : 0.0;
            acc[1] += on ? (double)u.y : 0.0;
            acc[2] += on ? (double)u.z : 0.0;
            acc[3] += on ? (double)u.w : 0.0;
            acc[4] += on ? (double)v.x : 0.0;
            acc[5] += on ? (double)v.y : 0.0;
            acc[6] += on ? (double)v.z : 0.0;
            acc[7] += on ? (double)v.w : 0.0;
        };
        auto fetch = [&](int64_t k, bool& on, float4& u, float4& v) {
            const RunDesc d = desc[k];
            on = (d.mask >> lane) & 1ull;
            const float4* row = reinterpret_cast<const float4*>(
                pb + (d.start + (on ? __popcll(d.mask & below) : 0)) * wb);
            u = row[0];
            v = row[1];
        };
        int64_t k = k0;
        for (; k + kRedUnroll <= k1; k += kRedUnroll) {
            bool on[kRedUnroll];
            float4 u[kRedUnroll], v[kRedUnroll];
#pragma unroll
            for (int i = 0; i < kRedUnroll; ++i) fetch(k + i, on[i], u[i], v[i]);
#pragma unroll
            for (int i = 0; i < kRedUnroll; ++i) add(on[i], u[i], v[i]);
        }
        for (; k < k1; ++k) {
            bool on;
            float4 u, v;
            fetch(k, on, u, v);
            add(on, u, v);
        }
        if (p < Mk) {
            double* r = red + (((int64_t)b * S + sl) * Mk + p) * l + c0;
#pragma unroll
            for (int c = 0; c < kRedCols; ++c)
                if (c < nc) r[c] = acc[c];
        }
    }
}

int hess_slices(int64_t Mk, int n_cu) {
    const int64_t G = (Mk + 63) / 64;
    const int64_t want = (16 * (int64_t)std::max(n_cu, 1) + G - 1) / std::max<int64_t>(G, 1);
    return (int)std::min<int64_t>(std::max<int64_t>(want, 1), 64);
}

// J^T weights of the Hessian product: W[b][p][k] = m_p C_p^2 scale sum_s red,
// split for the contraction (split_word).
__global__ void k_hess_weights(const double* __restrict__ red, int S, int64_t Mk, int l, int nb,
                               const double* __restrict__ C, const int32_t* __restrict__ kptr,
                               double scale, uint32_t* __restrict__ W, int64_t ldw) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nb * Mk * l) return;
    const int64_t k = i % l, p = (i / l) % Mk, b = i / (l * Mk);
    double t = 0.0;
    for (int s = 0; s < S; ++s) t += red[((b * S + s) * Mk + p) * l + k];
    const double m = (double)(kptr[p + 1] - kptr[p]);
    W[(b * Mk + p) * ldw + k] = split_word((float)(m * C[p] * C[p] * scale * t));
}

size_t jmb3_lds_bytes(int nb, int ntab, int tabfmt, int64_t n_tx) {
    const size_t tbytes = (size_t)nb * ntab * staged_entry_bytes(tabfmt);
    return ((tbytes + 15) & ~(size_t)15) + (size_t)n_tx * 64 * sizeof(float2) +
           4 * (size_t)nb * 64 * 36 * sizeof(uint32_t) + 64 * sizeof(int);
}

size_t psfb3_lds_bytes(int nb, int ntab, int tabfmt, int64_t n_tx);

template <int NB>
static hipError_t launch_hess_nb(hipStream_t s, int tabfmt, const ApplyArgs& a, const float* Q,
                                 int64_t ldq, int l, float* part, const int64_t* gptr,
                                 const void* desc, int S, double* red, const double* C,
                                 const int32_t* kptr, double scale, float* W, int64_t ldw,
                                 float* out) {
    if (!psf_weights_fit(a.M, ldw)) return hipErrorInvalidValue;
    const int wpb = a.waves_per_block;
    const unsigned nbat = (unsigned)((l + 32 * wpb - 1) / (32 * wpb));
    const unsigned grid = (unsigned)xcd_grid(a.n_act);
    auto run = [&](auto kern, size_t lds, auto... args) -> hipError_t {
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(kern, dim3(grid, nbat), dim3(64 * wpb), lds, s, a, args...);
        return hipGetLastError();
    };
    if (a.n_act == 0) return hipSuccess;
    const size_t lj = jmb3_lds_bytes(NB, a.ntab, tabfmt, a.n_tx);
    hipError_t e = hipErrorInvalidValue;
    switch (tabfmt) {
        case STAB_NODE32: e = run(k_jmb3<NB, float>, lj, Q, ldq, l, part); break;
        case STAB_NODE32Z: e = run(k_jmb3<NB, NodeZ>, lj, Q, ldq, l, part); break;
        case STAB_PAIR32: e = run(k_jmb3<NB, float2>, lj, Q, ldq, l, part); break;
        case STAB_BF16: e = run(k_jmb3<NB, uint32_t>, lj, Q, ldq, l, part); break;
    }
    if (e != hipSuccess) return e;
    const int64_t G = (a.M + 63) / 64;
    const int nz = (l + kRedCols - 1) / kRedCols;
    hipLaunchKernelGGL(k_reduce_cols,
                       dim3((unsigned)G, (unsigned)S,
                            (unsigned)((nz + kRedColWaves - 1) / kRedColWaves)),
                       dim3(64 * std::min(nz, kRedColWaves)), 0, s, part, a.nnz, l, gptr,
                       static_cast<const RunDesc*>(desc), a.M, NB, S, red);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nw = (int64_t)NB * a.M * l;
    hipLaunchKernelGGL(k_hess_weights, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, red, S,
                       a.M, l, NB, C, kptr, scale, reinterpret_cast<uint32_t*>(W), ldw);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lp = psfb3_lds_bytes(NB, a.ntab, tabfmt, a.n_tx);
    switch (tabfmt) {
        case STAB_NODE32: return run(k_psfb3<NB, float>, lp, (const float*)W, ldw, l, out);
        case STAB_NODE32Z: return run(k_psfb3<NB, NodeZ>, lp, (const float*)W, ldw, l, out);
        case STAB_PAIR32: return run(k_psfb3<NB, float2>, lp, (const float*)W, ldw, l, out);
        case STAB_BF16: return run(k_psfb3<NB, uint32_t>, lp, (const float*)W, ldw, l, out);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_hess_block(hipStream_t s, int tabfmt, const ApplyArgs& a, const float* Q,
                             int64_t ldq, int l, float* part, const int64_t* gptr,
                             const void* desc, int S, double* red, const double* C,
                             const int32_t* kptr, double scale, float* W, int64_t ldw,
                             float* out) {
    switch (a.nb) {
        case 1:
            return launch_hess_nb<1>(s, tabfmt, a, Q, ldq, l, part, gptr, desc, S, red, C, kptr,
                                     scale, W, ldw, out);
        case 2:
            return launch_hess_nb<2>(s, tabfmt, a, Q, ldq, l, part, gptr, desc, S, red, C, kptr,
                                     scale, W, ldw, out);
        case 3:
            return launch_hess_nb<3>(s, tabfmt, a, Q, ldq, l, part, gptr, desc, S, red, C, kptr,
                                     scale, W, ldw, out);
    }
    return hipErrorInvalidValue;
}

// ---- several right-hand sides at once (apply_J / apply_JT, n_rhs > 1)
//
// J Q for l model vectors: the Hessian's batched J (k_jmb3 partials, then
// k_reduce_cols' per-pair FP64 sums over the tiles), then every caller pair
// of kernel pair p gets C_p times its sum: out [l][nb][M].
__global__ void k_jbatch_out(const double* __restrict__ red, int S, int64_t Mk, int64_t M, int l,
                             int nb, const double* __restrict__ C,
                             const int32_t* __restrict__ kptr, const int32_t* __restrict__ kidx,
                             float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nb * Mk * l) return;
    const int64_t k = i % l, p = (i / l) % Mk, b = i / (l * Mk);
    double t = 0.0;
    for (int s = 0; s < S; ++s) t += red[((b * S + s) * Mk + p) * l + k];
    const float v = (float)(C[p] * t);
    for (int32_t j = kptr[p]; j < kptr[p + 1]; ++j) out[(k * nb + b) * M + kidx[j]] = v;
}

// J^T of l data vectors dT [l][nb][M]: the weight of kernel pair p for
// vector k is C_p times the sum of its caller pairs' data (FP64 sum, as the
// one-vector J^T), stored split for the BF16 matrix-core contraction.
__global__ void k_jtbatch_weights(const float* __restrict__ dT, int64_t Mk, int64_t M, int l,
                                  int nb, const double* __restrict__ C,
                                  const int32_t* __restrict__ kptr,
                                  const int32_t* __restrict__ kidx, uint32_t* __restrict__ W,
                                  int64_t ldw) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nb * Mk * l) return;
    const int64_t k = i % l, p = (i / l) % Mk, b = i / (l * Mk);
    double t = 0.0;
    for (int32_t j = kptr[p]; j < kptr[p + 1]; ++j) t += (double)dT[(k * nb + b) * M + kidx[j]];
    W[(b * Mk + p) * ldw + k] = split_word((float)(C[p] * t));
}

template <int NB>
static hipError_t launch_rhs_nb(hipStream_t s, int tabfmt, bool transpose, const ApplyArgs& a,
                                const float* in, int64_t ldq, int l, float* part,
                                const int64_t* gptr, const void* desc, int S, double* red,
                                const double* C, const int32_t* kptr, const int32_t* kidx,
                                int64_t M, uint32_t* W, int64_t ldw, float* out) {
    const int wpb = a.waves_per_block;
    const unsigned nbat = (unsigned)((l + 32 * wpb - 1) / (32 * wpb));
    const unsigned grid = (unsigned)xcd_grid(a.n_act);
    auto run = [&](auto kern, size_t lds, auto... args) -> hipError_t {
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(kern, dim3(grid, nbat), dim3(64 * wpb), lds, s, a, args...);
        return hipGetLastError();
    };
    const int64_t nw = (int64_t)NB * a.M * l;
    if (transpose) {
        if (!psf_weights_fit(a.M, ldw)) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_jtbatch_weights, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s,
                           in, a.M, M, l, NB, C, kptr, kidx, W, ldw);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || a.n_act == 0) return e;
        const size_t lp = psfb3_lds_bytes(NB, a.ntab, tabfmt, a.n_tx);
        switch (tabfmt) {
            case STAB_NODE32: return run(k_psfb3<NB, float>, lp, (const float*)W, ldw, l, out);
            case STAB_NODE32Z: return run(k_psfb3<NB, NodeZ>, lp, (const float*)W, ldw, l, out);
            case STAB_PAIR32: return run(k_psfb3<NB, float2>, lp, (const float*)W, ldw, l, out);
            case STAB_BF16: return run(k_psfb3<NB, uint32_t>, lp, (const float*)W, ldw, l, out);
        }
        return hipErrorInvalidValue;
    }
    hipError_t e = hipSuccess;
    if (a.n_act > 0) {
        const size_t lj = jmb3_lds_bytes(NB, a.ntab, tabfmt, a.n_tx);
        e = hipErrorInvalidValue;
        switch (tabfmt) {
            case STAB_NODE32: e = run(k_jmb3<NB, float>, lj, in, ldq, l, part); break;
            case STAB_NODE32Z: e = run(k_jmb3<NB, NodeZ>, lj, in, ldq, l, part); break;
            case STAB_PAIR32: e = run(k_jmb3<NB, float2>, lj, in, ldq, l, part); break;
            case STAB_BF16: e = run(k_jmb3<NB, uint32_t>, lj, in, ldq, l, part); break;
        }
        if (e != hipSuccess) return e;
        const int64_t G = (a.M + 63) / 64;
        const int nz = (l + kRedCols - 1) / kRedCols;
        hipLaunchKernelGGL(k_reduce_cols,
                           dim3((unsigned)G, (unsigned)S,
                                (unsigned)((nz + kRedColWaves - 1) / kRedColWaves)),
                           dim3(64 * std::min(nz, kRedColWaves)), 0, s, part, a.nnz, l, gptr,
                           static_cast<const RunDesc*>(desc), a.M, NB, S, red);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_jbatch_out, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, red, S,
                       a.M, M, l, NB, C, kptr, kidx, out);
    return hipGetLastError();
}

hipError_t launch_rhs_batch(hipStream_t s, int tabfmt, bool transpose, const ApplyArgs& a,
                            const float* in, int64_t ldq, int l, float* part, const int64_t* gptr,
                            const void* desc, int S, double* red, const double* C,
                            const int32_t* kptr, const int32_t* kidx, int64_t M, uint32_t* W,
                            int64_t ldw, float* out) {
    switch (a.nb) {
        case 1:
            return launch_rhs_nb<1>(s, tabfmt, transpose, a, in, ldq, l, part, gptr, desc, S, red,
                                    C, kptr, kidx, M, W, ldw, out);
        case 2:
            return launch_rhs_nb<2>(s, tabfmt, transpose, a, in, ldq, l, part, gptr, desc, S, red,
                                    C, kptr, kidx, M, W, ldw, out);
        case 3:
            return launch_rhs_nb<3>(s, tabfmt, transpose, a, in, ldq, l, part, gptr, desc, S, red,
                                    C, kptr, kidx, M, W, ldw, out);
    }
    return hipErrorInvalidValue;
}

size_t psfb3_lds_bytes(int nb, int ntab, int tabfmt, int64_t n_tx) {
    const size_t tbytes = (size_t)nb * ntab * staged_entry_bytes(tabfmt);
    const int ch = psfb3_chunk(nb);
    return std::max(((tbytes + 15) & ~(size_t)15) + (size_t)n_tx * 64 * sizeof(float2) +
                        2 * (2 * (size_t)nb * 64 * ((ch + 8) / 2) * sizeof(uint32_t) +
                             (size_t)ch * sizeof(int)),
                    kPsfOutLds);
}

size_t psf_lds_bytes(int nb, int ntab, int tabfmt, int64_t n_tx, bool b3) {
    if (b3 && nb <= 3) return psfb3_lds_bytes(nb, ntab, tabfmt, n_tx);
    const size_t tbytes = (size_t)nb * ntab * staged_entry_bytes(tabfmt);
    const int ch = nb == 1 ? psf_chunk<1>()
                 : (nb == 2 ? psf_chunk<2>() : (nb == 3 ? psf_chunk<3>() : psf_chunk<4>()));
    return std::max(((tbytes + 15) & ~(size_t)15) + (size_t)n_tx * 64 * sizeof(float2) +
                        2 * ((size_t)nb * ch * 64 * sizeof(float) + (size_t)ch * sizeof(int)),
                    kPsfOutLds);
}

template <int NB>
static hipError_t launch_psf_nb(hipStream_t s, int tabfmt, const ApplyArgs& a,
                                const int32_t* ptile, const int32_t* plane, const double* C,
                                const int32_t* kptr, double s2, float* W, int64_t ldw, int n,
                                float* out, const void* col_tab, bool b3) {
    // the weights (J e_k, cheap) always use the FP32 (h, slope) table, so a
    // BF16 table only enters through the contraction
    ApplyArgs ac = a;
    ac.tab = col_tab;
    // the split-BF16 contraction takes its weights already split
    const bool packed = b3 && NB <= 3;
    hipLaunchKernelGGL((k_psf_cols<NB, float2>), dim3((unsigned)n), dim3(64), 0, s, ac, ptile,
                       plane, C, kptr, s2, W, ldw, packed);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess || a.n_act == 0) return err;
    if (!psf_weights_fit(a.M, ldw)) return hipErrorInvalidValue;
    const int wpb = a.waves_per_block;
    const unsigned nbat = (unsigned)((n + 32 * wpb - 1) / (32 * wpb));
    const size_t lds = psf_lds_bytes(NB, a.ntab, tabfmt, a.n_tx, b3);
    auto run = [&](auto kern) -> hipError_t {
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
            if (e != hipSuccess) return e;
        }
        const unsigned grid = (unsigned)xcd_grid(a.n_act);
        hipLaunchKernelGGL(kern, dim3(grid, nbat), dim3(64 * wpb), lds, s, a, W, ldw, n, out);
        return hipGetLastError();
    };
    if constexpr (NB <= 3) {
        if (b3) {
            switch (tabfmt) {
                case STAB_NODE32: return run(k_psfb3<NB, float>);
                case STAB_NODE32Z: return run(k_psfb3<NB, NodeZ>);
                case STAB_PAIR32: return run(k_psfb3<NB, float2>);
                case STAB_BF16: return run(k_psfb3<NB, uint32_t>);
            }
            return hipErrorInvalidValue;
        }
    }
    switch (tabfmt) {
        case STAB_NODE32: return run(k_psf32<NB, float>);
        case STAB_NODE32Z: return run(k_psf32<NB, NodeZ>);
        case STAB_PAIR32: return run(k_psf32<NB, float2>);
        case STAB_BF16: return run(k_psf32<NB, uint32_t>);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_psf(hipStream_t s, int tabfmt, const ApplyArgs& a, const int32_t* ptile,
                      const int32_t* plane, const double* C, const int32_t* kptr, double s2,
                      float* W, int64_t ldw, int n, float* out, const void* col_tab, bool b3) {
    switch (a.nb) {
        case 1: return launch_psf_nb<1>(s, tabfmt, a, ptile, plane, C, kptr, s2, W, ldw, n, out,
                                        col_tab, b3);
        case 2: return launch_psf_nb<2>(s, tabfmt, a, ptile, plane, C, kptr, s2, W, ldw, n, out,
                                        col_tab, b3);
        case 3: return launch_psf_nb<3>(s, tabfmt, a, ptile, plane, C, kptr, s2, W, ldw, n, out,
                                        col_tab, b3);
        case 4: return launch_psf_nb<4>(s, tabfmt, a, ptile, plane, C, kptr, s2, W, ldw, n, out,
                                        col_tab, b3);
    }
    return hipErrorInvalidValue;
}



}  // namespace fftt
