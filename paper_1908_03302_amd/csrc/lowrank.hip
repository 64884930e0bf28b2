// Low-rank analysis of the Gauss-Newton Hessian H = J^T J / sigma^2 (Sec.
// II-E, eq. low_rank with Gamma_pr = I): the dense pieces of a randomized
// eigensolver on the matrix-free H, and the diagonals of the low-rank
// posterior covariance and resolution (eq. posterior_app / resolution_app).
//
// Blocks of vectors are stored one vector after another ([l][N], each
// vector contiguous), in the operator's precision; every inner product and
// small matrix is FP64.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace fftt {

namespace {

constexpr int kGJ = 32;              // rows per LDS stage
constexpr int64_t kGChunk = 4096;    // rows of one partial Gram block

// part[z][a][b] = sum_{j in chunk z} A[a][j] B[b][j] for one GT x GT tile
// of (a, b), GT = 16 RB; grid (ceil(la/GT), ceil(lb/GT), chunks), 256
// threads, each accumulating an RB x RB block (a = ta + 16 i, b = tb + 16 j)
// in registers, so one LDS read feeds RB / 2 FMAs.
template <int RB, class T>
__global__ __launch_bounds__(256) void k_gram_part(const T* __restrict__ A, int la,
                                                   const T* __restrict__ B, int lb, int64_t n,
                                                   double* __restrict__ part) {
    constexpr int GT = 16 * RB;
    __shared__ double sa[GT][kGJ + 1], sb[GT][kGJ + 1];
    const int a0 = blockIdx.x * GT, b0 = blockIdx.y * GT;
    const int64_t j0 = (int64_t)blockIdx.z * kGChunk;
    const int64_t j1 = min(n, j0 + kGChunk);
    const int ta = threadIdx.x / 16, tb = threadIdx.x % 16;
    double acc[RB][RB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < RB; ++j) acc[i][j] = 0.0;
    for (int64_t jb = j0; jb < j1; jb += kGJ) {
        for (int t = threadIdx.x; t < GT * kGJ; t += 256) {
            const int r = t / kGJ, col = t % kGJ;
            const int64_t j = jb + col;
            sa[r][col] = (a0 + r < la && j < j1) ? (double)A[(int64_t)(a0 + r) * n + j] : 0.0;
            sb[r][col] = (b0 + r < lb && j < j1) ? (double)B[(int64_t)(b0 + r) * n + j] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int col = 0; col < kGJ; ++col) {
            double av[RB], bv[RB];
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                av[i] = sa[ta + 16 * i][col];
                bv[i] = sb[tb + 16 * i][col];
            }
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int j = 0; j < RB; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            const int a = a0 + ta + 16 * i, b = b0 + tb + 16 * j;
            if (a < la && b < lb) part[((int64_t)blockIdx.z * la + a) * lb + b] = acc[i][j];
        }
}

// out[i] = sum_z part[z][i], one wave per i: lane t adds chunks t, t + 64,
// ... in order, then the 64 lane sums are added in a fixed tree.
__global__ __launch_bounds__(64) void k_gram_final(const double* __restrict__ part,
                                                   int64_t chunks, int64_t m,
                                                   double* __restrict__ out) {
    const int64_t i = blockIdx.x;
    const int lane = threadIdx.x;
    double s = 0.0;
    for (int64_t z = lane; z < chunks; z += 64) s += part[z * m + i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) out[i] = s;
}

using ConstD = const __attribute__((address_space(4))) double;

constexpr int kCombCols = 16;   // output vectors per pass over Y

// out[b][j] = sum_a Y[a][j] X[a][b] for b < m (X: [l][m] FP64, wave-uniform
// scalar loads); grid (ceil(n/256), ceil(m/kCombCols)).  Wider passes (one
// read of Y for up to 48 outputs) and requesting the next row of X ahead
// both measured slower.
template <class T>
__global__ __launch_bounds__(256) void k_combine(const T* __restrict__ Y, int l, int64_t n,
                                                 const double* X, int m, T* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int b0 = blockIdx.y * kCombCols;
    if (j >= n) return;
    ConstD* x = (ConstD*)X;
    double acc[kCombCols];
#pragma unroll
    for (int t = 0; t < kCombCols; ++t) acc[t] = 0.0;
    for (int a = 0; a < l; ++a) {
        const double y = (double)Y[(int64_t)a * n + j];
#pragma unroll
        for (int t = 0; t < kCombCols; ++t)
            acc[t] = fma(y, x[(int64_t)a * m + min(b0 + t, m - 1)], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < kCombCols; ++t)
        if (b0 + t < m) out[(int64_t)(b0 + t) * n + j] = (T)acc[t];
}

// var_j = (1 - sum_i d_i V[i][j]^2) / alpha, res_j = sum_i d_i V[i][j]^2.
template <class T>
__global__ void k_lowrank_diag(const T* __restrict__ V, int k, int64_t n,
                               const double* __restrict__ d, double inv_alpha,
                               T* __restrict__ var, T* __restrict__ res) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int i = 0; i < k; ++i) {
        const double v = (double)V[(int64_t)i * n + j];
        s = fma(d[i] * v, v, s);
    }
    if (var) var[j] = (T)((1.0 - s) * inv_alpha);
    if (res) res[j] = (T)s;
}

}  // namespace

hipError_t launch_gram(hipStream_t s, bool fp64, const void* A, int la, const void* B, int lb,
                       int64_t n, double* part, double* out) {
    const int64_t chunks = std::max<int64_t>((n + kGChunk - 1) / kGChunk, 1);
    // 48 x 48 tiles when they cover both sides (less padding for up to 48
    // vectors), else 64 x 64
    const int gt = std::max(la, lb) <= 48 ? 48 : 64;
    const dim3 grid((unsigned)((la + gt - 1) / gt), (unsigned)((lb + gt - 1) / gt),
                    (unsigned)chunks);
    if (gt == 48 && fp64)
        hipLaunchKernelGGL((k_gram_part<3, double>), grid, dim3(256), 0, s, (const double*)A,
                           la, (const double*)B, lb, n, part);
    else if (gt == 48)
        hipLaunchKernelGGL((k_gram_part<3, float>), grid, dim3(256), 0, s, (const float*)A, la,
                           (const float*)B, lb, n, part);
    else if (fp64)
        hipLaunchKernelGGL((k_gram_part<4, double>), grid, dim3(256), 0, s, (const double*)A,
                           la, (const double*)B, lb, n, part);
    else
        hipLaunchKernelGGL((k_gram_part<4, float>), grid, dim3(256), 0, s, (const float*)A, la,
                           (const float*)B, lb, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t m = (int64_t)la * lb;
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gram_final, dim3((unsigned)m), dim3(64), 0, s, part, chunks, m, out);
    return hipGetLastError();
}

size_t gram_part_doubles(int la, int lb, int64_t n) {
    return (size_t)std::max<int64_t>((n + kGChunk - 1) / kGChunk, 1) * la * lb;
}

hipError_t launch_combine(hipStream_t s, bool fp64, const void* Y, int l, int64_t n,
                          const double* X, int m, void* out) {
    if (n == 0 || m == 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256), (unsigned)((m + kCombCols - 1) / kCombCols));
    if (fp64)
        hipLaunchKernelGGL(k_combine<double>, grid, dim3(256), 0, s, (const double*)Y, l, n, X, m,
                           (double*)out);
    else
        hipLaunchKernelGGL(k_combine<float>, grid, dim3(256), 0, s, (const float*)Y, l, n, X, m,
                           (float*)out);
    return hipGetLastError();
}

hipError_t launch_lowrank_diag(hipStream_t s, bool fp64, const void* V, int k, int64_t n,
                               const double* d, double inv_alpha, void* var, void* res) {
    if (n == 0) return hipSuccess;
    const unsigned nblk = (unsigned)((n + 255) / 256);
    if (fp64)
        hipLaunchKernelGGL(k_lowrank_diag<double>, dim3(nblk), dim3(256), 0, s, (const double*)V,
                           k, n, d, inv_alpha, (double*)var, (double*)res);
    else
        hipLaunchKernelGGL(k_lowrank_diag<float>, dim3(nblk), dim3(256), 0, s, (const float*)V, k,
                           n, d, inv_alpha, (float*)var, (float*)res);
    return hipGetLastError();
}

// Symmetric eigen-decomposition by the cyclic Jacobi method (Golub & Van
// Loan, Sec. 8.5): plane rotations annihilate each off-diagonal entry in
// turn until the off-diagonal mass is negligible.  A [n][n] (overwritten),
// U [n][n] (columns = eigenvectors), w [n] eigenvalues, in descending order.
void jacobi_eigh(std::vector<double>& A, int n, std::vector<double>& w, std::vector<double>& U) {
    U.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) U[(size_t)i * n + i] = 1.0;
    auto at = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
    double total = 0.0;
    for (double v : A) total += v * v;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += at(i, j) * at(i, j);
        if (off <= 1e-30 * total || off == 0.0) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = at(p, q);
                if (apq == 0.0) continue;
                // rotation zeroing A[p][q]: tan of the angle from the
                // smaller root of t^2 + 2 theta t - 1 = 0
                const double theta = (at(q, q) - at(p, p)) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) /
                                 (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int r = 0; r < n; ++r) {   // A <- A G (columns p, q)
                    const double x = at(r, p), y = at(r, q);
                    at(r, p) = cs * x - sn * y;
                    at(r, q) = sn * x + cs * y;
                }
                for (int r = 0; r < n; ++r) {   // A <- G^T A (rows p, q)
                    const double x = at(p, r), y = at(q, r);
                    at(p, r) = cs * x - sn * y;
                    at(q, r) = sn * x + cs * y;
                }
                for (int r = 0; r < n; ++r) {   // U <- U G
                    double& x = U[(size_t)r * n + p];
                    double& y = U[(size_t)r * n + q];
                    const double ux = x, uy = y;
                    x = cs * ux - sn * uy;
                    y = sn * ux + cs * uy;
                }
            }
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return at(x, x) > at(y, y); });
    std::vector<double> Us((size_t)n * n);
    w.resize(n);
    for (int c = 0; c < n; ++c) {
        w[c] = at(idx[c], idx[c]);
        for (int r = 0; r < n; ++r) Us[(size_t)r * n + c] = U[(size_t)r * n + idx[c]];
    }
    U.swap(Us);
}

}  // namespace fftt
