// Compression basis for Section 7.B: an orthonormal basis Q of the dominant
// k-dimensional eigenspace of the Coulomb metric v, and S = Q^T v Q.
//
// Shifted subspace iteration: Q_{i+1} = orth((v + sigma 1) Q_i), starting
// from a counter-based random Q_0.  The shift keeps every iterate full rank
// (v itself may be rank deficient) without changing the eigenvectors or
// their order.  orth() is Cholesky QR on the rows of Q^T (every vector a
// contiguous row): G = Y^T Y, G = L L^T, Q^T = L^{-1} Y^T, done three times,
// the first with a small diagonal shift of G so that the factorisation cannot
// break down (shifted Cholesky QR3, Fukaya et al., SIAM J. Sci. Comput. 2020).
// Everything is a product on the matrix cores except the 64 x 64 diagonal
// blocks of the Cholesky factorisation.  The compressed interaction is then
// W = Q (1 - S chi_hat)^{-1} S Q^T with chi_hat = Q^T chi0 Q, which depends
// only on the subspace (any orthonormal basis of it gives the same W).
#include "gw_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace gwk {

hipError_t launch_dgemm(hipStream_t st, int M, int N, int K, double alpha, const double *A, int64_t lda, int64_t sA,
                        const double *B, int64_t ldb, int64_t sB, double beta, double *C, int64_t ldc, int64_t sC,
                        int batch);

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

// Cholesky of the w x w diagonal block at (p, p) of G (row-major, ld k) in
// LDS, after adding shift_rel * (*tr) to its diagonal.  Writes L back into
// the lower triangle of the block, L^{-1} to Li and L^{-T} to LiT (64 x 64,
// zero outside w x w).  A pivot not above floor_rel * (*tr) (and positive)
// sets *bad (the rows were linearly dependent, or not finite) and is replaced
// by 1.
__global__ __launch_bounds__(256) void k_potf2(int k, int p, int w, double *G, const double *tr, double shift_rel,
                                               double floor_rel, double *Li, double *LiT, int *bad) {
    __shared__ double a[64][65];
    __shared__ double inv[64][65];
    const int t = threadIdx.x;
    const double shift = shift_rel * *tr, floor_piv = floor_rel * *tr;
    for (int e = t; e < 64 * 64; e += 256) {
        const int i = e >> 6, j = e & 63;
        double x = 0.0;
        if (i < w && j <= i) {
            x = G[(int64_t)(p + i) * k + p + j];
            if (i == j) x += shift;
        }
        a[i][j] = x;
        inv[i][j] = 0.0;
    }
    __syncthreads();
    for (int c = 0; c < w; ++c) {
        const double d = a[c][c];
        const bool ok = d > floor_piv && d > 0.0;
        const double piv = ok ? sqrt(d) : 1.0;
        __syncthreads();
        if (t == 0) {
            a[c][c] = piv;
            if (!ok) *bad = 1;
        }
        for (int i = c + 1 + t; i < w; i += 256) a[i][c] /= piv;
        __syncthreads();
        const int m = w - c - 1;
        for (int e = t; e < m * m; e += 256) {
            const int i = c + 1 + e / m, j = c + 1 + e % m;
            if (j <= i) a[i][j] -= a[i][c] * a[j][c];
        }
        __syncthreads();
    }
    // L^{-1}, column j by thread j (forward substitution on e_j)
    if (t < w) {
        const int j = t;
        for (int i = j; i < w; ++i) {
            double s = (i == j) ? 1.0 : 0.0;
            for (int q = j; q < i; ++q) s -= a[i][q] * inv[q][j];
            inv[i][j] = s / a[i][i];
        }
    }
    __syncthreads();
    for (int e = t; e < 64 * 64; e += 256) {
        const int i = e >> 6, j = e & 63;
        const bool in = i < w && j < w;
        if (in && j <= i) G[(int64_t)(p + i) * k + p + j] = a[i][j];
        Li[i * 64 + j] = in ? inv[i][j] : 0.0;
        LiT[j * 64 + i] = in ? inv[i][j] : 0.0;
    }
}

// dst[c * ldd + r] = src[r * lds + c] for r < rows, c < cols
__global__ __launch_bounds__(256) void k_transpose_ld(int rows, int cols, const double *src, int64_t lds, double *dst,
                                                      int64_t ldd) {
    __shared__ double tt[32][33];
    const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int q = ty; q < 32; q += 8)
        if (r0 + q < rows && c0 + tx < cols) tt[q][tx] = src[(int64_t)(r0 + q) * lds + c0 + tx];
    __syncthreads();
    for (int q = ty; q < 32; q += 8)
        if (c0 + q < cols && r0 + tx < rows) dst[(int64_t)(c0 + q) * ldd + r0 + tx] = tt[tx][q];
}

__global__ void k_zero_i(int *p) { *p = 0; }

hipError_t transpose_ld(hipStream_t st, int rows, int cols, const double *src, int64_t lds, double *dst,
                        int64_t ldd) {
    dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
    hipLaunchKernelGGL(k_transpose_ld, grid, dim3(256), 0, st, rows, cols, src, lds, dst, ldd);
    return hipGetLastError();
}

struct CholWs {
    double *G, *Li, *LiT, *T, *tr;
    int *bad;
};

// G (k x k, row-major) = L L^T in place (lower triangle), blocked by 64:
// diagonal block in LDS, then L21 = G21 L11^{-T} and G22 -= L21 L21^T on the
// matrix cores.  The L21 product runs in place: each 64-row band of the
// output reads its own w input columns completely before writing.
hipError_t potrf(hipStream_t st, int k, double shift_rel, const CholWs &c, double floor_rel = 0.0) {
    hipError_t e;
    for (int p = 0; p < k; p += 64) {
        const int w = std::min(64, k - p), rest = k - p - w;
        double *li = c.Li + (int64_t)(p / 64) * 4096, *lit = c.LiT + (int64_t)(p / 64) * 4096;
        hipLaunchKernelGGL(k_potf2, dim3(1), dim3(256), 0, st, k, p, w, c.G, c.tr, shift_rel, floor_rel, li, lit,
                           c.bad);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (rest > 0) {
            double *G21 = c.G + (int64_t)(p + w) * k + p;
            if ((e = launch_dgemm(st, rest, w, w, 1.0, G21, k, 0, lit, 64, 0, 0.0, G21, k, 0, 1)) != hipSuccess)
                return e;
            if ((e = transpose_ld(st, rest, w, G21, k, c.T, rest)) != hipSuccess) return e;
            if ((e = launch_dgemm(st, rest, rest, w, -1.0, G21, k, 0, c.T, rest, 0, 1.0, G21 + w, k, 0, 1)) !=
                hipSuccess)
                return e;
        }
    }
    return hipSuccess;
}

// Yt (k x n) <- L^{-1} Yt, blocked forward substitution (right-looking).
hipError_t trsm_lower(hipStream_t st, int k, int n, const CholWs &c, double *Yt) {
    hipError_t e;
    for (int p = 0; p < k; p += 64) {
        const int w = std::min(64, k - p), rest = k - p - w;
        double *Yp = Yt + (int64_t)p * n;
        // in place: a single 64-row band, each column tile reads all w rows first
        if ((e = launch_dgemm(st, w, n, w, 1.0, c.Li + (int64_t)(p / 64) * 4096, 64, 0, Yp, n, 0, 0.0, Yp, n, 0, 1)) !=
            hipSuccess)
            return e;
        if (rest > 0 && (e = launch_dgemm(st, rest, n, w, -1.0, c.G + (int64_t)(p + w) * k + p, k, 0, Yp, n, 0, 1.0,
                                          Yp + (int64_t)w * n, n, 0, 1)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// One Cholesky QR pass on the rows of Yt (k x n); Y is n x k scratch.
hipError_t cholqr(hipStream_t st, int k, int n, double *Yt, double *Y, double shift_rel, const CholWs &c) {
    hipError_t e;
    if ((e = transpose_ld(st, k, n, Yt, n, Y, k)) != hipSuccess) return e;
    if ((e = launch_dgemm(st, k, k, n, 1.0, Yt, n, 0, Y, k, 0, 0.0, c.G, k, 0, 1)) != hipSuccess) return e;
    if (shift_rel > 0) {
        hipLaunchKernelGGL(k_trace, dim3(1), dim3(1024), 0, st, c.G, k, c.tr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = potrf(st, k, shift_rel, c)) != hipSuccess) return e;
    return trsm_lower(st, k, n, c, Yt);
}

// Orthonormalise the rows of Yt in place: shifted Cholesky QR, then two plain
// passes.  The shift 11 (n k + k (k + 1)) u tr(G) bounds the one the method
// prescribes (tr(G) >= |Y|_2^2).
hipError_t orth_rows(hipStream_t st, int k, int n, double *Yt, double *Y, const CholWs &c) {
    const double u = 1.1102230246251565e-16;
    const double shift_rel = 11.0 * ((double)n * k + (double)k * (k + 1)) * u;
    hipError_t e = cholqr(st, k, n, Yt, Y, shift_rel, c);
    if (e != hipSuccess) return e;
    if ((e = cholqr(st, k, n, Yt, Y, 0.0, c)) != hipSuccess) return e;
    return cholqr(st, k, n, Yt, Y, 0.0, c);
}

}  // namespace

size_t compress_work_doubles(int n, int k) {
    const size_t nblk = (size_t)(k + 63) / 64;
    return 3 * (size_t)k * n + (size_t)k * k + 2 * nblk * 4096 + 64;
}

// work: compress_work_doubles(n, k).  Returns hipErrorUnknown if a Cholesky
// pivot was not positive (not expected: the shift keeps every iterate full
// rank, so only a non-finite v gets there).
hipError_t compress_basis(hipStream_t st, int n, int k, const double *v, double *Q_out, double *S_out, double *work,
                          int iters) {
    const int64_t kn = (int64_t)k * n;
    const int64_t nblk = (k + 63) / 64;
    double *Qt = work;
    double *Yt = Qt + kn;
    double *T = Yt + kn;  // n x k scratch, then Qt v
    CholWs c;
    c.G = T + kn;
    c.Li = c.G + (int64_t)k * k;
    c.LiT = c.Li + nblk * 4096;
    c.tr = c.LiT + nblk * 4096;
    c.bad = (int *)(c.tr + 2);
    double *vtr = c.tr + 4;
    c.T = T;
    unsigned blocks = (unsigned)std::min<int64_t>((kn + 255) / 256, 8192);
    hipLaunchKernelGGL(k_rand, dim3(blocks), dim3(256), 0, st, Yt, kn, 0x5eedull);
    hipLaunchKernelGGL(k_trace, dim3(1), dim3(1024), 0, st, v, n, vtr);
    hipLaunchKernelGGL(k_zero_i, dim3(1), dim3(1), 0, st, c.bad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double trace = 0;
    e = hipMemcpyAsync(&trace, vtr, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    const double sigma = (trace > 0 ? trace : 1.0) * 1e-6;
    if ((e = orth_rows(st, k, n, Yt, T, c)) != hipSuccess) return e;
    std::swap(Qt, Yt);
    for (int it = 0; it < iters; ++it) {
        // Yt = Qt v + sigma Qt  ((v + sigma) Q)^T, v symmetric
        hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, st, Qt, Yt, kn);
        if ((e = launch_dgemm(st, k, n, n, 1.0, Qt, n, 0, v, n, 0, sigma, Yt, n, 0, 1)) != hipSuccess) return e;
        if ((e = orth_rows(st, k, n, Yt, T, c)) != hipSuccess) return e;
        std::swap(Qt, Yt);
    }
    // S = Qt v Qt^T, Q = Qt^T
    if ((e = launch_dgemm(st, k, n, n, 1.0, Qt, n, 0, v, n, 0, 0.0, T, n, 0, 1)) != hipSuccess) return e;
    if ((e = transpose_ld(st, k, n, Qt, n, Q_out, k)) != hipSuccess) return e;
    if ((e = launch_dgemm(st, k, k, n, 1.0, T, n, 0, Q_out, k, 0, 0.0, S_out, k, 0, 1)) != hipSuccess) return e;
    int hb = 0;
    e = hipMemcpyAsync(&hb, c.bad, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    return hb ? hipErrorUnknown : hipSuccess;
}

namespace {

// X[mu][j0 + j] = P[mu][src[j0 + j] - base] for j < ncols (selected pair columns)
__global__ void k_gather_cols(int ncols, int64_t ldp, const double *__restrict__ P, const int32_t *__restrict__ src,
                              int64_t base, int j0, double *__restrict__ X, int64_t ldx) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int mu = blockIdx.y;
    if (j >= ncols) return;
    X[(int64_t)mu * ldx + j0 + j] = P[(int64_t)mu * ldp + (src[j0 + j] - base)];
}

}  // namespace

hipError_t launch_gather_cols(hipStream_t st, int rows, int ncols, int64_t ldp, const double *P, const int32_t *src,
                              int64_t base, int j0, double *X, int64_t ldx) {
    if (ncols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)((ncols + 255) / 256), (unsigned)rows), dim3(256), 0, st, ncols,
                       ldp, P, src, base, j0, X, ldx);
    return hipGetLastError();
}

size_t pair_basis_work_doubles(int n, int nr, int k) {
    const size_t nblk = (size_t)(k + 63) / 64;
    return 2 * (size_t)n * nr + (size_t)nr * nr + (size_t)nr * k + (size_t)k * k + compress_work_doubles(nr, k) +
           3 * (size_t)n * k + 2 * nblk * 4096 + (size_t)64 * std::max(n, k) + 64;
}

// Section 7.A subspace from its generators X [n][nr] (pair vectors below the
// energy threshold): g = X^T v X (eq. projector0); Qg [nr][k] an orthonormal
// basis of the dominant k-dimensional eigenspace of g (shifted subspace
// iteration, as for v) and Sg = Qg^T g Qg; with Sg = L L^T,
// Z = X Qg L^{-T} is orthonormal in the Coulomb metric (Z^T v Z = 1,
// eq. global-basis-orthogonality) and spans the same space as the paper's
// X xi / sqrt(lambda) (eq. subspace).  Also U = v Z and, if R is not null,
// R = v - U U^T.  Returns hipErrorUnknown if the iteration lost a direction
// or the k-th eigenvalue of g is below 1e-10 of the trace of Sg (k exceeds
// the rank of the generators).
hipError_t pair_basis(hipStream_t st, int n, int nr, int k, const double *v, const double *X, double *Z, double *U,
                      double *R, double *work, int iters) {
    hipError_t e;
    const int64_t nblk = (k + 63) / 64;
    double *Xt = work;                         // [nr][n]
    double *T1 = Xt + (int64_t)nr * n;         // [n][nr], later reused
    double *g = T1 + (int64_t)n * nr;          // [nr][nr]
    double *Qg = g + (int64_t)nr * nr;         // [nr][k]
    double *Sg = Qg + (int64_t)nr * k;         // [k][k]
    double *cw = Sg + (int64_t)k * k;          // compress_basis work
    double *Y = cw + compress_work_doubles(nr, k);  // [n][k]
    double *Yt = Y + (int64_t)n * k;           // [k][n]
    double *Ut = Yt + (int64_t)k * n;          // [k][n]
    CholWs c;
    c.G = Sg;
    c.Li = Ut + (int64_t)k * n;
    c.LiT = c.Li + nblk * 4096;
    c.T = c.LiT + nblk * 4096;                 // 64 x max(n, k)
    c.tr = c.T + (int64_t)64 * std::max(n, k);
    c.bad = (int *)(c.tr + 2);
    // g = X^T (v X)
    if ((e = launch_dgemm(st, n, nr, n, 1.0, v, n, 0, X, nr, 0, 0.0, T1, nr, 0, 1)) != hipSuccess) return e;
    if ((e = transpose_ld(st, n, nr, X, nr, Xt, n)) != hipSuccess) return e;
    if ((e = launch_dgemm(st, nr, nr, n, 1.0, Xt, n, 0, T1, nr, 0, 0.0, g, nr, 0, 1)) != hipSuccess) return e;
    if ((e = compress_basis(st, nr, k, g, Qg, Sg, cw, iters)) != hipSuccess) return e;
    // Y = X Qg; Sg = L L^T (pivots must exceed 1e-10 tr Sg); Z^T = L^{-1} Y^T
    if ((e = launch_dgemm(st, n, k, nr, 1.0, X, nr, 0, Qg, k, 0, 0.0, Y, k, 0, 1)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_i, dim3(1), dim3(1), 0, st, c.bad);
    hipLaunchKernelGGL(k_trace, dim3(1), dim3(1024), 0, st, Sg, k, c.tr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = potrf(st, k, 0.0, c, 1e-10)) != hipSuccess) return e;
    if ((e = transpose_ld(st, n, k, Y, k, Yt, n)) != hipSuccess) return e;
    if ((e = trsm_lower(st, k, n, c, Yt)) != hipSuccess) return e;
    if ((e = transpose_ld(st, k, n, Yt, n, Z, k)) != hipSuccess) return e;
    // U = v Z; R = v - U U^T
    if ((e = launch_dgemm(st, n, k, n, 1.0, v, n, 0, Z, k, 0, 0.0, U, k, 0, 1)) != hipSuccess) return e;
    if (R) {
        if ((e = transpose_ld(st, n, k, U, k, Ut, n)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_copy, dim3((unsigned)std::min<int64_t>(((int64_t)n * n + 255) / 256, 8192)), dim3(256),
                           0, st, v, R, (int64_t)n * n);
        if ((e = launch_dgemm(st, n, n, k, -1.0, U, k, 0, Ut, n, 0, 1.0, R, n, 0, 1)) != hipSuccess) return e;
    }
    int hb = 0;
    if ((e = hipMemcpyAsync(&hb, c.bad, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    return hb ? hipErrorUnknown : hipSuccess;
}

}  // namespace gwk
