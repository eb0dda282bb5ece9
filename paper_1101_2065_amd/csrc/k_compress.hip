// Compression basis for Section 7.B: an orthonormal basis Q of the dominant
// k-dimensional eigenspace of the Coulomb metric v, and S = Q^T v Q.
//
// Shifted subspace iteration: Q_{i+1} = orth((v + sigma 1) Q_i), starting
// from a counter-based random Q_0.  The shift keeps every iterate full rank
// (v itself may be rank deficient) without changing the eigenvectors or
// their order.  Orthonormalisation is classical Gram-Schmidt with one full
// re-orthogonalisation (CGS2), row by row on Q^T (so every vector is a
// contiguous row).  The compressed interaction is then
// W = Q (1 - S chi_hat)^{-1} S Q^T with chi_hat = Q^T chi0 Q, which depends
// only on the subspace (any orthonormal basis of it gives the same W).
#include "gw_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace gwk {

hipError_t launch_dgemm(hipStream_t st, int M, int N, int K, double alpha, const double *A, int64_t lda, int64_t sA,
                        const double *B, int64_t ldb, int64_t sB, double beta, double *C, int64_t ldc, int64_t sC,
                        int batch);
hipError_t launch_transpose_d(hipStream_t st, int rows, int cols, const double *src, double *dst);

namespace {

// SplitMix64 (Steele, Lea, Flood 2014) of (seed, index) -> uniform [-1, 1)
__device__ inline double rnd(uint64_t seed, uint64_t i) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void k_rand(double *p, int64_t n, uint64_t seed) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = rnd(seed, (uint64_t)i);
}

__global__ void k_copy(const double *s, double *d, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = s[i];
}

// trace of v (for the shift), single workgroup
__global__ __launch_bounds__(1024) void k_trace(const double *v, int n, double *out) {
    __shared__ double red[16];
    double s = 0;
    for (int i = threadIdx.x; i < n; i += 1024) s += v[(int64_t)i * n + i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int q = 0; q < 16; ++q) t += red[q];
        *out = t;
    }
}

// d[j] = Qt[j] . y for j < c (one workgroup per j); also |y|^2 into d[c] by workgroup c
__global__ __launch_bounds__(256) void k_dots(const double *Qt, const double *y, int n, int c, double *d) {
    __shared__ double red[4];
    const int j = blockIdx.x;
    const double *q = (j < c) ? Qt + (int64_t)j * n : y;
    double s = 0;
    for (int i = threadIdx.x; i < n; i += 256) s += q[i] * y[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) d[j] = red[0] + red[1] + red[2] + red[3];
}

// y -= sum_j d[j] Qt[j]  (thread per element); stores |y|^2 partials
__global__ __launch_bounds__(256) void k_project(const double *Qt, double *y, int n, int c, const double *d,
                                                 double *nrm2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    double v = 0;
    if (i < n) {
        v = y[i];
        for (int j = 0; j < c; ++j) v -= d[j] * Qt[(int64_t)j * n + i];
        y[i] = v;
    }
    double s = v * v;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) atomicAdd(nrm2, s);
}

// Qt[c] = y / |y|.  If the projection removed almost everything
// (|y| <= 1e-10 of the norm before projection) the basis would lose a
// direction: *bad is set and the caller reports the failure.
__global__ __launch_bounds__(256) void k_normalise(const double *y, int n, const double *nrm2, const double *nrm0,
                                                   double *Qrow, int *bad) {
    const double nr = sqrt(*nrm2), n0 = sqrt(*nrm0);
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (!(nr > 1e-10 * n0) || !(nr > 0.0)) {
        if (i == 0) *bad = 1;
        return;
    }
    if (i < n) Qrow[i] = y[i] / nr;
}

__global__ void k_zero_d(double *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

}  // namespace

// Orthonormalise the rows of Yt (k x n) into Qt (k x n) by CGS2.
// work: k + 4 doubles; bad: device flag set if a row lost its direction.
static hipError_t orth_rows(hipStream_t st, int k, int n, double *Yt, double *Qt, double *work, int *bad) {
    double *d = work;  // [k]
    double *nrm2 = work + k + 1;
    double *nrm0 = work + k + 2;
    const unsigned gb = (unsigned)((n + 255) / 256);
    for (int c = 0; c < k; ++c) {
        double *y = Yt + (int64_t)c * n;
        hipLaunchKernelGGL(k_dots, dim3(1), dim3(256), 0, st, Qt, y, n, 0, nrm0);
        for (int pass = 0; pass < 2; ++pass) {
            if (c > 0) hipLaunchKernelGGL(k_dots, dim3(c), dim3(256), 0, st, Qt, y, n, c, d);
            hipLaunchKernelGGL(k_zero_d, dim3(1), dim3(64), 0, st, nrm2, 1);
            hipLaunchKernelGGL(k_project, dim3(gb), dim3(256), 0, st, Qt, y, n, c, d, nrm2);
        }
        hipLaunchKernelGGL(k_normalise, dim3(gb), dim3(256), 0, st, y, n, nrm2, nrm0, Qt + (int64_t)c * n, bad);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// work: 3 k n + k + 16 doubles.  Returns hipErrorUnknown if the iteration
// lost a direction (not expected: the shift keeps every iterate full rank).
hipError_t compress_basis(hipStream_t st, int n, int k, const double *v, double *Q_out, double *S_out, double *work,
                          int iters) {
    // work layout: Qt [k][n], Yt [k][n], T [k][n], misc [k + 16]
    double *Qt = work;
    double *Yt = Qt + (int64_t)k * n;
    double *T = Yt + (int64_t)k * n;
    double *misc = T + (int64_t)k * n;
    double *tr = misc + k + 4;
    int *bad = (int *)(misc + k + 5);
    const int64_t kn = (int64_t)k * n;
    unsigned blocks = (unsigned)std::min<int64_t>((kn + 255) / 256, 8192);
    hipLaunchKernelGGL(k_rand, dim3(blocks), dim3(256), 0, st, Yt, kn, 0x5eedull);
    hipLaunchKernelGGL(k_trace, dim3(1), dim3(1024), 0, st, v, n, tr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double trace = 0;
    e = hipMemcpyAsync(&trace, tr, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    const double sigma = (trace > 0 ? trace : 1.0) * 1e-6;
    hipLaunchKernelGGL(k_zero_d, dim3(1), dim3(64), 0, st, (double *)bad, 1);
    e = orth_rows(st, k, n, Yt, Qt, misc, bad);
    if (e != hipSuccess) return e;
    for (int it = 0; it < iters; ++it) {
        // Yt = Qt v + sigma Qt  ((v + sigma) Q)^T, v symmetric
        hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, st, Qt, Yt, kn);
        e = launch_dgemm(st, k, n, n, 1.0, Qt, n, 0, v, n, 0, sigma, Yt, n, 0, 1);
        if (e != hipSuccess) return e;
        e = orth_rows(st, k, n, Yt, Qt, misc, bad);
        if (e != hipSuccess) return e;
    }
    // S = Qt v Qt^T, Q = Qt^T
    e = launch_dgemm(st, k, n, n, 1.0, Qt, n, 0, v, n, 0, 0.0, T, n, 0, 1);
    if (e != hipSuccess) return e;
    e = launch_transpose_d(st, k, n, Qt, Q_out);
    if (e != hipSuccess) return e;
    e = launch_dgemm(st, k, k, n, 1.0, T, n, 0, Q_out, k, 0, 0.0, S_out, k, 0, 1);
    if (e != hipSuccess) return e;
    int hb = 0;
    e = hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    return hb ? hipErrorUnknown : hipSuccess;
}

}  // namespace gwk
