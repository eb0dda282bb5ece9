// Exact part of the chi0 build on gfx950: pair vertex, mesh bins, bin-sorted
// pair order and the int64 spectral histogram.  Compiled with
// -ffp-contract=off: every product and sum is rounded on its own, in the
// same order as the definition, so the results are bit-reproducible.
//
// Paper: Foerster, Koval, Sanchez-Portal, arXiv:1101.2065.
//   pair vertex       Section 7.A, V_mu^{EF} = X_a^E V_mu^{ab} X_b^F
//   spectral function Section 5.A eq. chi_by_spectra (odd extension a(-s) = -a(s))
//   mesh              Section 5 and 5.B
#include "gw_internal.h"
#include "gw_prof.h"

#include <hip/hip_runtime.h>
#include <math.h>

namespace gwk {

namespace {

// Magic constant 1.5 * 2^52: for |x| < 2^51, fl(x + M) holds round-to-nearest-even(x)
// in its low mantissa bits, so bits(fl(x + M)) - bits(M) = RNE(x) as int64.
constexpr double kMagic = 6755399441055744.0;
constexpr uint64_t kMagicBits = 0x4338000000000000ull;

__device__ inline void pair_bin(const double *eig, int n_occ, int E, int Fp, int kbits, int *m,
                                double *frac) {
#pragma clang fp contract(off)
    double d = __dsub_rn(eig[n_occ + Fp], eig[E]);
    double x = ldexp(d, kbits);  // exact: the mesh spacing is 2^-kbits
    double fm = floor(x);
    *m = (int)fm;
    *frac = __dsub_rn(x, fm);
}

// ------------------------------------------------------------------ pair vertex
// One workgroup per (product mu, chunk of 128 empty states F').  Each thread
// owns one F': T[a] = sum_b V^{ab} X_b^F (b ascending), then for every occupied
// E, P = sum_a X_a^E T[a] (a ascending); products and sums rounded separately,
// the same order the oracle uses, so the result is bit-identical.
template <int NMAX>
__global__ __launch_bounds__(128) void k_pairvec(int n_orb, int n_occ, int n_blk, const double *__restrict__ X,
                                                 const int32_t *__restrict__ blk_prod,
                                                 const int32_t *__restrict__ blk_orb,
                                                 const int32_t *__restrict__ orb_idx,
                                                 const int64_t *__restrict__ blk_val,
                                                 const double *__restrict__ vals, int e0, int ecnt, int64_t ldp,
                                                 double *__restrict__ P) {
#pragma clang fp contract(off)
    __shared__ double Vs[NMAX * NMAX];
    __shared__ int Os[NMAX];
    const int mu = blockIdx.x;
    const int n_virt = n_orb - n_occ;
    // block of mu: largest b with blk_prod[b] <= mu
    int lo = 0, hi = n_blk - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (blk_prod[mid] <= mu) lo = mid; else hi = mid - 1;
    }
    const int b = lo;
    const int n = blk_orb[b + 1] - blk_orb[b];
    const double *Vm = vals + blk_val[b] + (int64_t)(mu - blk_prod[b]) * n * n;
    for (int i = threadIdx.x; i < n * n; i += blockDim.x) Vs[i] = Vm[i];
    for (int i = threadIdx.x; i < n; i += blockDim.x) Os[i] = orb_idx[blk_orb[b] + i];
    __syncthreads();
    const int f = blockIdx.y * 128 + threadIdx.x;
    if (f >= n_virt) return;
    double T[NMAX];
#pragma unroll
    for (int a = 0; a < NMAX; ++a) T[a] = 0.0;
    for (int bb = 0; bb < n; ++bb) {
        const double xb = X[(int64_t)Os[bb] * n_orb + n_occ + f];
#pragma unroll
        for (int a = 0; a < NMAX; ++a)
            if (a < n) T[a] = __dadd_rn(T[a], __dmul_rn(Vs[a * n + bb], xb));
    }
    // occupied states e0 .. e0+ecnt-1 go to columns (E - e0) * n_virt + F' of row mu
    double *Prow = P + (int64_t)mu * ldp + f - (int64_t)e0 * n_virt;
    for (int E = e0; E < e0 + ecnt; ++E) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < NMAX; ++a)
            if (a < n) acc = __dadd_rn(acc, __dmul_rn(X[(int64_t)Os[a] * n_orb + E], T[a]));
        Prow[(int64_t)E * n_virt] = acc;
    }
}

// ------------------------------------------------------------------ bins and order
// lo[E][m] = number of F' whose bin is < m (bins are non-decreasing in F'
// because the eigenvalues are sorted).
__global__ void k_lobound(int n_orb, int n_occ, const double *__restrict__ eig, int kbits, int nhb,
                          int32_t *__restrict__ lo) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)n_occ * (nhb + 1);
    if (idx >= total) return;
    const int E = (int)(idx / (nhb + 1));
    const int m = (int)(idx % (nhb + 1));
    const int n_virt = n_orb - n_occ;
    int a = 0, bnd = n_virt;  // first F' with bin >= m
    while (a < bnd) {
        int mid = (a + bnd) >> 1;
        int mm;
        double fr;
        pair_bin(eig, n_occ, E, mid, kbits, &mm, &fr);
        if (mm < m) a = mid + 1; else bnd = mid;
    }
    lo[idx] = a;
}

// Per-bin counts, per-row offsets and the exclusive scan over bins.  Bins that
// can hold pairs are 0..nhb-2 (the upper neighbour m+1 must exist).
__global__ __launch_bounds__(1024) void k_binscan(int n_occ, int nhb, int64_t n_pairs,
                                                  const int32_t *__restrict__ lo,
                                                  int32_t *__restrict__ rowoff,
                                                  int32_t *__restrict__ binoff,
                                                  int64_t *__restrict__ stat) {
    extern __shared__ int32_t cnt[];
    for (int m = threadIdx.x; m < nhb - 1; m += blockDim.x) {
        int32_t run = 0;
        for (int E = 0; E < n_occ; ++E) {
            rowoff[(int64_t)E * nhb + m] = run;
            run += lo[(int64_t)E * (nhb + 1) + m + 1] - lo[(int64_t)E * (nhb + 1) + m];
        }
        cnt[m] = run;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t acc = 0;
        for (int m = 0; m < nhb - 1; ++m) {
            binoff[m] = acc;
            acc += cnt[m];
        }
        binoff[nhb - 1] = acc;
        stat[0] = acc;
        stat[1] = n_pairs - acc;
    }
}

__global__ void k_sortpairs(int n_orb, int n_occ, const double *__restrict__ eig, int kbits, int nhb,
                            const int32_t *__restrict__ lo, const int32_t *__restrict__ rowoff,
                            const int32_t *__restrict__ binoff, int32_t *__restrict__ perm,
                            double *__restrict__ fsort) {
    const int n_virt = n_orb - n_occ;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)n_occ * n_virt) return;
    const int E = (int)(p / n_virt);
    const int Fp = (int)(p % n_virt);
    int m;
    double fr;
    pair_bin(eig, n_occ, E, Fp, kbits, &m, &fr);
    if (m + 1 >= nhb) return;  // beyond the mesh: dropped
    const int64_t pos = (int64_t)binoff[m] + rowoff[(int64_t)E * nhb + m] + (Fp - lo[(int64_t)E * (nhb + 1) + m]);
    perm[pos] = (int32_t)p;
    fsort[pos] = fr;
}

__global__ void k_gather(int64_t n_pairs, const double *__restrict__ P, const int32_t *__restrict__ perm,
                         const int64_t *__restrict__ stat, double *__restrict__ Ps) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= stat[0]) return;
    Ps[(int64_t)r * n_pairs + i] = P[(int64_t)r * n_pairs + perm[i]];
}

__global__ void k_absmax(const double *__restrict__ P, int64_t n, uint64_t *__restrict__ dst) {
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, fabs(P[i]));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) atomicMax((unsigned long long *)dst, (unsigned long long)__double_as_longlong(m));
}

__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// s = min(61 - c - 2e, 50 - 2e), vmax < 2^e, 2*n_pairs < 2^c, clamped to
// [-200, 960]; an explicit request is honoured only if it is not larger.
__global__ void k_fracbits(const uint64_t *vmax_bits, int64_t n_pairs, int requested, int32_t *s_out) {
    const double vmax = __longlong_as_double((long long)*vmax_bits);
    int e = 0;
    (void)frexp(vmax, &e);
    const uint64_t two_n = (uint64_t)(2 * n_pairs);
    const int c = two_n ? 64 - __clzll((long long)two_n) : 0;
    int s = min(61 - c - 2 * e, 50 - 2 * e);
    s = max(-200, min(960, s));
    if (requested >= 0 && requested < s) s = requested;
    *s_out = s;
}

// ------------------------------------------------------------------ histogram
// H[m][t] for t = packed(mu <= nu).  Workgroup = 64x64 (mu, nu) tile and one
// slice of the bin range; 256 threads, each owning a 4x4 register tile
// (mu = mu0 + ty + 16 i, nu = nu0 + tx + 16 j).  Pairs arrive sorted by bin, so
// each thread keeps two running int64 sums per entry for the current bin:
//   A = sum RNE(2^s V_mu V_nu),  B = sum RNE(fl(fl(V_mu 2^s frac) V_nu))
// (held with the magic offset, removed at the flush) and emits
//   H[m] += 2 (A - B) + 2 B(m-1),
// i.e. the lower share of bin m plus the upper share carried from bin m-1.
// Integer additions are exact and associative, so the result does not depend
// on the launch shape or the order of the pairs.
constexpr int HT = 64;  // tile edge
constexpr int HC = 32;  // pairs per staged chunk

__global__ __launch_bounds__(256) void k_hist(int n, int64_t ldp, const double *__restrict__ Ps,
                                              const double *__restrict__ fsort,
                                              const int32_t *__restrict__ binoff,
                                              const int64_t *__restrict__ stat,
                                              const int32_t *__restrict__ s_dev, int nhb,
                                              unsigned long long *__restrict__ H, int64_t n_upper,
                                              int ntiles, int splits, int bin_lo, int bin_hi) {
#pragma clang fp contract(off)
    // rows padded by one value: the staging stores walk down a column
    __shared__ double Pm[HC][HT + 1];
    __shared__ double Pn[HC][HT + 1];
    __shared__ double wv[HC];
    // decode (ti <= tj) from blockIdx.x, row-major over the upper triangle of tiles
    int t = blockIdx.x;
    int ti = 0;
    while (t >= ntiles - ti) {
        t -= ntiles - ti;
        ++ti;
    }
    const int tj = ti + t;
    const int mu0 = ti * HT, nu0 = tj * HT;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    (void)stat;  // the kept-pair count is binoff[nhb - 1]
    const int s = *s_dev;
    const double twos = ldexp(1.0, s);
    // bin slice [mb, me) of this split: only pairs whose lower bin lies in
    // [bin_lo, bin_hi), cut at bin boundaries into `splits` runs of about
    // equal length (so a launch over a few bins still fills the grid)
    const int q = blockIdx.y;
    auto first_bin = [&](int64_t target) {
        int a = 0, b = nhb - 1;  // binoff[nhb-1] = the kept pairs >= target
        while (a < b) {
            int mid = (a + b) >> 1;
            if (binoff[mid] >= target) b = mid; else a = mid + 1;
        }
        return a;
    };
    const int64_t plo = binoff[bin_lo], span = binoff[bin_hi] - plo;
    const int mb = max(bin_lo, (q == 0) ? bin_lo : first_bin(plo + (span * q) / splits));
    const int me = min(bin_hi, (q == splits - 1) ? bin_hi : first_bin(plo + (span * (q + 1)) / splits));
    if (mb >= me) return;

    uint64_t A[4][4], B[4][4], Bp[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) A[i][j] = B[i][j] = Bp[i][j] = 0;
    bool valid[4][4];
    int64_t tidx[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int mu = mu0 + ty + 16 * i, nu = nu0 + tx + 16 * j;
            valid[i][j] = (mu < n) && (nu < n) && (mu <= nu);
            tidx[i][j] = (int64_t)mu * n - ((int64_t)mu * (mu - 1)) / 2 + (nu - mu);
        }

    for (int m = mb; m < me; ++m) {
        const int64_t p0 = binoff[m], p1 = binoff[m + 1];
        for (int64_t c0 = p0; c0 < p1; c0 += HC) {
            const int cnt = (int)min((int64_t)HC, p1 - c0);
            __syncthreads();
            for (int r = threadIdx.x; r < HC * HT; r += 256) {
                const int row = r / HC, col = r % HC;
                double a = 0.0, b = 0.0;
                if (col < cnt) {
                    if (mu0 + row < n) a = Ps[(int64_t)(mu0 + row) * ldp + c0 + col];
                    if (nu0 + row < n) b = Ps[(int64_t)(nu0 + row) * ldp + c0 + col];
                }
                Pm[col][row] = a;
                Pn[col][row] = b;
            }
            if (threadIdx.x < HC) wv[threadIdx.x] = threadIdx.x < cnt ? ldexp(fsort[c0 + threadIdx.x], s) : 0.0;
            __syncthreads();
            for (int pp = 0; pp < cnt; ++pp) {
                const double w = wv[pp];
                double u[4], y[4], vn[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const double vm = Pm[pp][ty + 16 * i];
                    u[i] = __dmul_rn(vm, twos);
                    y[i] = __dmul_rn(vm, w);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) vn[j] = Pn[pp][tx + 16 * j];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const double x = __dadd_rn(__dmul_rn(u[i], vn[j]), kMagic);
                        const double z = __dadd_rn(__dmul_rn(y[i], vn[j]), kMagic);
                        A[i][j] += (uint64_t)__double_as_longlong(x);
                        B[i][j] += (uint64_t)__double_as_longlong(z);
                    }
            }
        }
        const uint64_t off = (uint64_t)(p1 - p0) * kMagicBits;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint64_t val = 2ull * (A[i][j] - B[i][j] + Bp[i][j]);
                if (valid[i][j] && val != 0ull)
                    atomicAdd(&H[(int64_t)m * n_upper + tidx[i][j]], (unsigned long long)val);
                Bp[i][j] = B[i][j] - off;
                A[i][j] = 0;
                B[i][j] = 0;
            }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t val = 2ull * Bp[i][j];
            if (valid[i][j] && val != 0ull) atomicAdd(&H[(int64_t)me * n_upper + tidx[i][j]], (unsigned long long)val);
        }
}

}  // namespace


hipError_t launch_pairvec(hipStream_t st, int n_orb, int n_occ, int n_prod, int n_blk, const double *X,
                          const int32_t *blk_prod, const int32_t *blk_orb, const int32_t *orb_idx,
                          const int64_t *blk_val, const double *vals, int max_o, int e0, int ecnt, int64_t ldp,
                          double *P) {
    const int n_virt = n_orb - n_occ;
    dim3 grid(n_prod, (n_virt + 127) / 128);
    if (max_o <= 16)
        hipLaunchKernelGGL(k_pairvec<16>, grid, dim3(128), 0, st, n_orb, n_occ, n_blk, X, blk_prod, blk_orb,
                           orb_idx, blk_val, vals, e0, ecnt, ldp, P);
    else if (max_o <= 32)
        hipLaunchKernelGGL(k_pairvec<32>, grid, dim3(128), 0, st, n_orb, n_occ, n_blk, X, blk_prod, blk_orb,
                           orb_idx, blk_val, vals, e0, ecnt, ldp, P);
    else if (max_o <= 64)
        hipLaunchKernelGGL(k_pairvec<64>, grid, dim3(128), 0, st, n_orb, n_occ, n_blk, X, blk_prod, blk_orb,
                           orb_idx, blk_val, vals, e0, ecnt, ldp, P);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_pair_sort(hipStream_t st, int n_orb, int n_occ, const double *eig, int kbits, int nhb,
                            int32_t *lo, int32_t *rowoff, int32_t *binoff, int32_t *perm, double *fsort,
                            int64_t *stat) {
    const int64_t tot = (int64_t)n_occ * (nhb + 1);
    hipLaunchKernelGGL(k_lobound, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n_orb, n_occ, eig,
                       kbits, nhb, lo);
    const int64_t n_pairs = (int64_t)n_occ * (n_orb - n_occ);
    hipLaunchKernelGGL(k_binscan, dim3(1), dim3(1024), (size_t)nhb * sizeof(int32_t), st, n_occ, nhb, n_pairs,
                       lo, rowoff, binoff, stat);
    hipLaunchKernelGGL(k_sortpairs, dim3((unsigned)((n_pairs + 255) / 256)), dim3(256), 0, st, n_orb, n_occ,
                       eig, kbits, nhb, lo, rowoff, binoff, perm, fsort);
    return hipGetLastError();
}

hipError_t launch_gather(hipStream_t st, int rows, int64_t n_pairs, const double *P, const int32_t *perm,
                         const int64_t *stat, double *Ps) {
    dim3 grid((unsigned)((n_pairs + 255) / 256), rows);
    hipLaunchKernelGGL(k_gather, grid, dim3(256), 0, st, n_pairs, P, perm, stat, Ps);
    return hipGetLastError();
}

hipError_t launch_absmax(hipStream_t st, const double *P, int64_t n, uint64_t *dst) {
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, dst, (int64_t)1, (uint64_t)0);
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_absmax, dim3((unsigned)blocks), dim3(256), 0, st, P, n, dst);
    return hipGetLastError();
}

hipError_t launch_fracbits(hipStream_t st, const uint64_t *vmax_bits, int64_t n_pairs, int requested,
                           int32_t *s_out) {
    hipLaunchKernelGGL(k_fracbits, dim3(1), dim3(1), 0, st, vmax_bits, n_pairs, requested, s_out);
    return hipGetLastError();
}

hipError_t launch_fill_u64(hipStream_t st, uint64_t *p, int64_t n, uint64_t value) {
    GW_DEFER(launch_fill_u64(st, p, n, value));
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, st, p, n, value);
    return hipGetLastError();
}

hipError_t launch_hist(hipStream_t st, int n, int64_t n_pairs_cap, const double *Ps, const double *fsort,
                       const int32_t *binoff, const int64_t *stat, const int32_t *s_dev, int nhb, int64_t *H,
                       int splits, int bin_lo, int bin_hi, bool clear) {
    const int64_t n_upper = (int64_t)n * (n + 1) / 2;
    if (bin_hi < 0 || bin_hi > nhb - 1) bin_hi = nhb - 1;
    if (bin_lo < 0 || bin_lo > bin_hi) return hipErrorInvalidValue;
    // only rows [bin_lo, bin_hi] can receive weight; only they are cleared
    // (clear = false: the caller cleared them, and consecutive ranges add up)
    if (clear) {
        hipError_t e = launch_fill_u64(st, (uint64_t *)H + (int64_t)bin_lo * n_upper,
                                       (int64_t)(bin_hi - bin_lo + 1) * n_upper, 0);
        if (e != hipSuccess) return e;
    }
    const int ntiles = (n + HT - 1) / HT;
    const int ntp = ntiles * (ntiles + 1) / 2;
    if (splits < 1) splits = 1;
    ProfScope ps(st, "hist", (double)n_pairs_cap * n_upper,
                 8.0 * (double)n_pairs_cap * n + 8.0 * (bin_hi - bin_lo + 1) * n_upper);
    hipLaunchKernelGGL(k_hist, dim3(ntp, splits), dim3(256), 0, st, n, n_pairs_cap, Ps, fsort, binoff, stat, s_dev,
                       nhb, (unsigned long long *)H, n_upper, ntiles, splits, bin_lo, bin_hi);
    return hipGetLastError();
}

namespace {
__global__ void k_sub_i64(const int64_t *__restrict__ a, int64_t *__restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i] - b[i];
}
}  // namespace

// b = a - b (exact integer histogram difference)
hipError_t launch_sub_i64(hipStream_t st, const int64_t *a, int64_t *b, int64_t n) {
    const int64_t blocks = std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 8192);
    hipLaunchKernelGGL(k_sub_i64, dim3((unsigned)blocks), dim3(256), 0, st, a, b, n);
    return hipGetLastError();
}

}  // namespace gwk
