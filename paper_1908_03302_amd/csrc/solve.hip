// Regularised least squares on the matrix-free operators (Sec. II-D,
// eq. leastSquare_misfit1 / leastSquare_misfit with Gamma_n = sigma^2 I and
// Gamma_pr = I) and Hessian point-spread functions (eq. resolution_2).
//
// All vectors stay on the device.  Inner products are accumulated in FP64 in
// a fixed order (per-block partials, then one block), and the scalar
// recurrences of CGLS / LSQR run in a one-thread kernel on device-resident
// scalars, so an iteration issues no host synchronisation.
#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace fftt {

namespace {

constexpr int kDotBlocks = 512;
constexpr int kDotThreads = 256;

template <class T>
__global__ __launch_bounds__(kDotThreads) void k_dot_part(const T* __restrict__ a,
                                                          const T* __restrict__ b, int64_t n,
                                                          double* __restrict__ part) {
    __shared__ double s[kDotThreads];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kDotThreads)
        acc += (double)a[i] * (double)b[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kDotThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// out[slot] = scale * sum(part[0..n))
__global__ __launch_bounds__(kDotThreads) void k_dot_final(const double* __restrict__ part, int n,
                                                           double* __restrict__ sc, int slot,
                                                           double scale) {
    __shared__ double s[kDotThreads];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kDotThreads) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kDotThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sc[slot] = scale * s[0];
}

// y = cy * y + cx * x, where cy = ay (* sc[sy] if sy >= 0), cx likewise.
template <class T>
__global__ void k_axpby(T* y, const T* x, int64_t n, double ay, int sy,
                        double ax, int sx, const double* __restrict__ sc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double cy = sy >= 0 ? ay * sc[sy] : ay;
    const double cx = sx >= 0 ? ax * sc[sx] : ax;
    y[i] = (T)(cy * (double)y[i] + cx * (double)x[i]);
}

// z = ax * x + ay * y (host constants)
template <class T>
__global__ void k_lin2(T* z, const T* x, const T* y,
                       int64_t n, double ax, double ay) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    z[i] = (T)(ax * (double)x[i] + ay * (double)(y ? y[i] : (T)0));
}

// ---- scalar recurrences (slots of the device scalar array) ----
enum Slot {
    GAMMA = 0, DELTA_Q = 1, DELTA_P = 2, STEP = 3, BETA = 4, MISFIT = 5, GAMMA0 = 6, GNEW = 7,
    // LSQR
    L_BETA = 8, L_ALPHA = 9, L_RHOBAR = 10, L_PHIBAR = 11, L_PHI_RHO = 12, L_THETA_RHO = 13,
    L_XX = 14, L_INV_BETA = 15, L_INV_ALPHA = 16, L_NEG_BETA = 17, L_NEG_ALPHA = 18, L_RES2 = 19,
    NSLOTS = 24
};

__global__ void k_cgls_step(double* sc, double alpha_reg) {
    // a = gamma / (|q|^2 + alpha |p|^2)
    const double d = sc[DELTA_Q] + alpha_reg * sc[DELTA_P];
    sc[STEP] = d > 0.0 ? sc[GAMMA] / d : 0.0;
}

__global__ void k_cgls_beta(double* sc) {
    const double g = sc[GAMMA];
    sc[BETA] = g > 0.0 ? sc[GNEW] / g : 0.0;
    sc[GAMMA] = sc[GNEW];
}

// After u <- A v - alpha u: beta = |u| (slot holds |u|^2), scale factors.
__global__ void k_lsqr_beta(double* sc) {
    const double b = sqrt(fmax(sc[L_BETA], 0.0));
    sc[L_BETA] = b;
    sc[L_INV_BETA] = b > 0.0 ? 1.0 / b : 0.0;
    sc[L_NEG_BETA] = -b;
}

// After v <- A^T u - beta v: alpha = |v|; then the two plane rotations.
__global__ void k_lsqr_alpha_rot(double* sc, double damp, int first) {
    const double a = sqrt(fmax(sc[L_ALPHA], 0.0));
    sc[L_ALPHA] = a;
    sc[L_INV_ALPHA] = a > 0.0 ? 1.0 / a : 0.0;
    sc[L_NEG_ALPHA] = -a;
    if (first) {  // initial: rhobar = alpha1, phibar = beta1
        sc[L_RHOBAR] = a;
        sc[L_PHIBAR] = sc[L_BETA];
        return;
    }
    const double beta = sc[L_BETA];
    const double rhobar = sc[L_RHOBAR];
    double phibar = sc[L_PHIBAR];
    const double rhobar1 = hypot(rhobar, damp);
    const double c1 = rhobar1 > 0.0 ? rhobar / rhobar1 : 1.0;
    const double s1 = rhobar1 > 0.0 ? damp / rhobar1 : 0.0;
    const double psi = s1 * phibar;   // part of the residual moved into the damping block
    sc[L_RES2] += psi * psi;
    phibar *= c1;
    const double rho = hypot(rhobar1, beta);
    const double c = rho > 0.0 ? rhobar1 / rho : 1.0;
    const double s = rho > 0.0 ? beta / rho : 0.0;
    const double theta = s * a;
    sc[L_RHOBAR] = -c * a;
    const double phi = c * phibar;
    sc[L_PHIBAR] = s * phibar;
    sc[L_PHI_RHO] = rho > 0.0 ? phi / rho : 0.0;
    sc[L_THETA_RHO] = rho > 0.0 ? -theta / rho : 0.0;
    // |A x - b|^2 = phibar^2 + sum psi^2 - damp^2 |x|^2 is formed on the host
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

template <class T>
static hipError_t dot(hipStream_t s, const T* a, const T* b, int64_t n, double* part, double* sc,
                      int slot, double scale) {
    hipLaunchKernelGGL(k_dot_part<T>, dim3(kDotBlocks), dim3(kDotThreads), 0, s, a, b, n, part);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kDotThreads), 0, s, part, kDotBlocks, sc, slot,
                       scale);
    return hipGetLastError();
}

template <class T>
static hipError_t axpby(hipStream_t s, T* y, const T* x, int64_t n, double ay, int sy, double ax,
                        int sx, const double* sc) {
    hipLaunchKernelGGL(k_axpby<T>, dim3(nblk(n)), dim3(256), 0, s, y, x, n, ay, sy, ax, sx, sc);
    return hipGetLastError();
}

template <class T>
static hipError_t lin2(hipStream_t s, T* z, const T* x, const T* y, int64_t n, double ax,
                       double ay) {
    hipLaunchKernelGGL(k_lin2<T>, dim3(nblk(n)), dim3(256), 0, s, z, x, y, n, ax, ay);
    return hipGetLastError();
}

hipError_t solver_dot(hipStream_t s, bool fp64, const void* a, const void* b, int64_t n,
                      double* part, double* sc, int slot, double scale) {
    return fp64 ? dot(s, (const double*)a, (const double*)b, n, part, sc, slot, scale)
                : dot(s, (const float*)a, (const float*)b, n, part, sc, slot, scale);
}

hipError_t solver_axpby(hipStream_t s, bool fp64, void* y, const void* x, int64_t n, double ay,
                        int sy, double ax, int sx, const double* sc) {
    return fp64 ? axpby(s, (double*)y, (const double*)x, n, ay, sy, ax, sx, sc)
                : axpby(s, (float*)y, (const float*)x, n, ay, sy, ax, sx, sc);
}

hipError_t solver_lin2(hipStream_t s, bool fp64, void* z, const void* x, const void* y, int64_t n,
                       double ax, double ay) {
    return fp64 ? lin2(s, (double*)z, (const double*)x, (const double*)y, n, ax, ay)
                : lin2(s, (float*)z, (const float*)x, (const float*)y, n, ax, ay);
}

hipError_t solver_cgls_step(hipStream_t s, double* sc, double alpha_reg) {
    hipLaunchKernelGGL(k_cgls_step, dim3(1), dim3(1), 0, s, sc, alpha_reg);
    return hipGetLastError();
}

hipError_t solver_cgls_beta(hipStream_t s, double* sc) {
    hipLaunchKernelGGL(k_cgls_beta, dim3(1), dim3(1), 0, s, sc);
    return hipGetLastError();
}

hipError_t solver_lsqr_beta(hipStream_t s, double* sc) {
    hipLaunchKernelGGL(k_lsqr_beta, dim3(1), dim3(1), 0, s, sc);
    return hipGetLastError();
}

hipError_t solver_lsqr_alpha_rot(hipStream_t s, double* sc, double damp, int first) {
    hipLaunchKernelGGL(k_lsqr_alpha_rot, dim3(1), dim3(1), 0, s, sc, damp, first);
    return hipGetLastError();
}

// ---- Jacobi preconditioner ----

// minv = 1 / (scale * diag + alpha) (0 where that is not positive)
template <class T>
__global__ void k_jacobi(T* __restrict__ minv, const float* __restrict__ diag, int64_t n,
                         double scale, double alpha) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double d = scale * (double)diag[i] + alpha;
    minv[i] = (T)(d > 0.0 ? 1.0 / d : 0.0);
}

// z = a * b elementwise
template <class T>
__global__ void k_mul(T* __restrict__ z, const T* __restrict__ a, const T* __restrict__ b,
                      int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = a[i] * b[i];
}

hipError_t solver_jacobi(hipStream_t s, bool fp64, void* minv, const float* diag, int64_t n,
                         double scale, double alpha) {
    if (fp64)
        hipLaunchKernelGGL(k_jacobi<double>, dim3(nblk(n)), dim3(256), 0, s, (double*)minv, diag,
                           n, scale, alpha);
    else
        hipLaunchKernelGGL(k_jacobi<float>, dim3(nblk(n)), dim3(256), 0, s, (float*)minv, diag,
                           n, scale, alpha);
    return hipGetLastError();
}

hipError_t solver_mul(hipStream_t s, bool fp64, void* z, const void* a, const void* b,
                      int64_t n) {
    if (fp64)
        hipLaunchKernelGGL(k_mul<double>, dim3(nblk(n)), dim3(256), 0, s, (double*)z,
                           (const double*)a, (const double*)b, n);
    else
        hipLaunchKernelGGL(k_mul<float>, dim3(nblk(n)), dim3(256), 0, s, (float*)z,
                           (const float*)a, (const float*)b, n);
    return hipGetLastError();
}

// ---- point-spread functions ----

// dc = e_v (1 m/s at voxel v): zero fill then one element.
template <class T>
__global__ void k_unit(T* __restrict__ x, int64_t n, int64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = (T)(i == v ? 1.0 : 0.0);
}

constexpr int kFillCols = 8;   // vectors per wavefront of k_fill_runs

// Zeroes, in each of n vectors of length N, the index ranges [runs[2 r],
// runs[2 r] + runs[2 r + 1]): one wavefront per (range, kFillCols vectors),
// 16-byte stores where range and vector starts are multiples of 4 and the
// output is 16-byte aligned.
__global__ __launch_bounds__(64) void k_fill_runs(float* __restrict__ out, int64_t N, int n,
                                                  const int64_t* __restrict__ runs) {
    const int64_t st = runs[2 * (int64_t)blockIdx.x], len = runs[2 * (int64_t)blockIdx.x + 1];
    const int k0 = (int)blockIdx.y * kFillCols, k1 = min(n, k0 + kFillCols);
    const bool vec = ((st | len | N) & 3) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0;
    for (int k = k0; k < k1; ++k) {
        float* __restrict__ o = out + (int64_t)k * N + st;
        if (vec) {
            for (int64_t i = threadIdx.x; i < len / 4; i += 64)
                reinterpret_cast<float4*>(o)[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        } else {
            for (int64_t i = threadIdx.x; i < len; i += 64) o[i] = 0.0f;
        }
    }
}

hipError_t fill_runs(hipStream_t s, float* out, int64_t N, int n, const int64_t* runs,
                     int64_t nruns) {
    if (nruns == 0 || n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_runs, dim3((unsigned)nruns, (unsigned)((n + kFillCols - 1) / kFillCols)),
                       dim3(64), 0, s, out, N, n, runs);
    return hipGetLastError();
}

hipError_t solver_unit(hipStream_t s, bool fp64, void* x, int64_t n, int64_t v) {
    if (fp64)
        hipLaunchKernelGGL(k_unit<double>, dim3(nblk(n)), dim3(256), 0, s, (double*)x, n, v);
    else
        hipLaunchKernelGGL(k_unit<float>, dim3(nblk(n)), dim3(256), 0, s, (float*)x, n, v);
    return hipGetLastError();
}

}  // namespace fftt
