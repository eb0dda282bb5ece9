// Blocked right-looking LU with partial pivoting, batched over frequencies,
// and the matching solve, for W(w) = (1 - v chi0(w))^{-1} v (Section 2 eq.
// Coulombscreening; the inversion is the O(N^3) step the paper's Sections 1
// and 7.B point to).
//
// Panel width 64 (inside 256-wide blocks, see getrf_impl).  Per panel: one
// workgroup per frequency factors the
// (n - kb) x 64 panel column by column (pivot = largest |re| + |im|, ties to
// the lowest row), composes the 64 row exchanges into one list of
// (destination, source) rows, and inverts the 64x64 unit-lower L11 and the
// upper U11 in LDS.  The row exchanges are then applied to the rest of the
// matrix in one pass, U12 = L11^{-1} A12 and the trailing update
// A22 -= L21 U12 run on the MFMA GEMM.  The solve uses the stored inverses the
// same way, so every O(N^3) flop of factor and solve is an MFMA product.
#include "gw_internal.h"
#include "gw_prof.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace gwk {

hipError_t launch_zgemm(hipStream_t st, int M, int N, int K, double alpha, const zdbl *A, int64_t lda, int64_t sA,
                        const zdbl *B, int64_t ldb, int64_t sB, double beta, zdbl *C, int64_t ldc, int64_t sC,
                        int batch);
hipError_t launch_cgemm(hipStream_t st, int M, int N, int K, float alpha, const zflt *A, int64_t lda, int64_t sA,
                        const zflt *B, int64_t ldb, int64_t sB, float beta, zflt *C, int64_t ldc, int64_t sC,
                        int batch);

namespace {

constexpr int NB = 64;         // panel width
constexpr int SWP = 1 + 4 * NB;  // per-frequency swap list: count, dst[2NB], src[2NB]

template <typename T>
struct Cx {
    T re, im;
};
template <typename T>
__device__ inline Cx<T> cmul(Cx<T> a, Cx<T> b) {
    return Cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ inline Cx<T> crcp(Cx<T> a) {
    const T d = a.re * a.re + a.im * a.im;
    return Cx<T>{a.re / d, -a.im / d};
}

template <typename T>
__global__ __launch_bounds__(512) void k_getf2(int n, int kb, int w, Cx<T> *A, int64_t sA, int32_t *ipiv,
                                               Cx<T> *Linv, Cx<T> *Uinv, int nblk, Cx<T> *S, int32_t *swp,
                                               int32_t *info) {
    __shared__ Cx<T> Ts[NB][NB];
    __shared__ Cx<T> Xs[NB][NB];
    __shared__ Cx<T> urow[NB];
    __shared__ T red_v[8];
    __shared__ int red_i[8];
    __shared__ int lpiv[NB];
    __shared__ int piv_s;
    __shared__ int zero_s;
    __shared__ int rows[2 * NB], cont[2 * NB];
    __shared__ Cx<T> dinv[NB];

    const int b = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    A += (int64_t)b * sA;
    ipiv += (int64_t)b * n;
    S += (int64_t)b * NB * n;
    swp += (int64_t)b * SWP;
    Linv += ((int64_t)b * nblk + kb / NB) * NB * NB;
    Uinv += ((int64_t)b * nblk + kb / NB) * NB * NB;
    const int m = n - kb;

    for (int64_t idx = tid; idx < (int64_t)m * w; idx += 512) {
        const int i = (int)(idx / w), c = (int)(idx % w);
        S[(int64_t)c * m + i] = A[(int64_t)(kb + i) * n + kb + c];
    }
    __syncthreads();

    for (int j = 0; j < w; ++j) {
        const Cx<T> *col = S + (int64_t)j * m;
        T best = T(-1);
        int bi = m;
        for (int i = j + tid; i < m; i += 512) {
            const Cx<T> z = col[i];
            const T v = fabs(z.re) + fabs(z.im);
            if (v > best) {
                best = v;
                bi = i;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const T ov = __shfl_xor(best, off);
            const int oi = __shfl_xor(bi, off);
            if (ov > best || (ov == best && oi < bi)) {
                best = ov;
                bi = oi;
            }
        }
        if (lane == 0) {
            red_v[wave] = best;
            red_i[wave] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            T bv = red_v[0];
            int bx = red_i[0];
            for (int q = 1; q < 8; ++q)
                if (red_v[q] > bv || (red_v[q] == bv && red_i[q] < bx)) {
                    bv = red_v[q];
                    bx = red_i[q];
                }
            if (bx >= m) bx = j;
            piv_s = bx;
            lpiv[j] = bx;
            zero_s = (bv == T(0));
            if (bv == T(0) && info[b] == 0) info[b] = kb + j + 1;
        }
        __syncthreads();
        const int piv = piv_s;
        if (piv != j) {
            for (int c = tid; c < w; c += 512) {
                Cx<T> *pc = S + (int64_t)c * m;
                const Cx<T> t = pc[j];
                pc[j] = pc[piv];
                pc[piv] = t;
            }
        }
        __syncthreads();
        if (!zero_s) {
            const Cx<T> inv = crcp(S[(int64_t)j * m + j]);
            if (tid > j && tid < w) urow[tid] = S[(int64_t)tid * m + j];
            __syncthreads();
            for (int i = j + 1 + tid; i < m; i += 512) {
                Cx<T> *pj = S + (int64_t)j * m;
                const Cx<T> l = cmul(pj[i], inv);
                pj[i] = l;
                for (int c = j + 1; c < w; ++c) {
                    Cx<T> *pc = S + (int64_t)c * m;
                    const Cx<T> u = urow[c];
                    const Cx<T> x = pc[i];
                    pc[i] = Cx<T>{x.re - (l.re * u.re - l.im * u.im), x.im - (l.re * u.im + l.im * u.re)};
                }
            }
        }
        __syncthreads();
    }

    // write the factored panel back, pivots as global rows
    for (int64_t idx = tid; idx < (int64_t)m * w; idx += 512) {
        const int i = (int)(idx / w), c = (int)(idx % w);
        A[(int64_t)(kb + i) * n + kb + c] = S[(int64_t)c * m + i];
    }
    if (tid < w) ipiv[kb + tid] = kb + lpiv[tid];
    // compose the row exchanges: new row dst = old row src
    if (tid == 0) {
        int nt = 0;
        for (int j = 0; j < w; ++j) {
            const int r1 = j, r2 = lpiv[j];
            if (r1 == r2) continue;
            int i1 = -1, i2 = -1;
            for (int t = 0; t < nt; ++t) {
                if (rows[t] == r1) i1 = t;
                if (rows[t] == r2) i2 = t;
            }
            if (i1 < 0) {
                rows[nt] = r1;
                cont[nt] = r1;
                i1 = nt++;
            }
            if (i2 < 0) {
                rows[nt] = r2;
                cont[nt] = r2;
                i2 = nt++;
            }
            const int t = cont[i1];
            cont[i1] = cont[i2];
            cont[i2] = t;
        }
        swp[0] = nt;
        for (int t = 0; t < nt; ++t) {
            swp[1 + t] = kb + rows[t];
            swp[1 + 2 * NB + t] = kb + cont[t];
        }
    }
    // diagonal block into LDS (row-major), zero padded
    for (int idx = tid; idx < NB * NB; idx += 512) {
        const int i = idx / NB, c = idx % NB;
        Ts[i][c] = (i < w && c < w) ? S[(int64_t)c * m + i] : Cx<T>{T(0), T(0)};
        Xs[i][c] = Cx<T>{T(0), T(0)};
    }
    __syncthreads();
    // L11^{-1}: unit lower, column c by forward substitution
    if (tid < w) {
        const int c = tid;
        Xs[c][c] = Cx<T>{T(1), T(0)};
        for (int i = c + 1; i < w; ++i) {
            T sr = 0, si = 0;
            for (int k = c; k < i; ++k) {
                const Cx<T> l = Ts[i][k], x = Xs[k][c];
                sr += l.re * x.re - l.im * x.im;
                si += l.re * x.im + l.im * x.re;
            }
            Xs[i][c] = Cx<T>{-sr, -si};
        }
    }
    if (tid < w) dinv[tid] = crcp(Ts[tid][tid]);
    __syncthreads();
    for (int idx = tid; idx < NB * NB; idx += 512) {
        Linv[idx] = Xs[idx / NB][idx % NB];
        Xs[idx / NB][idx % NB] = Cx<T>{T(0), T(0)};
    }
    __syncthreads();
    // U11^{-1}: upper, column c by back substitution
    if (tid < w) {
        const int c = tid;
        Xs[c][c] = dinv[c];
        for (int i = c - 1; i >= 0; --i) {
            T sr = 0, si = 0;
            for (int k = i + 1; k <= c; ++k) {
                const Cx<T> u = Ts[i][k], x = Xs[k][c];
                sr += u.re * x.re - u.im * x.im;
                si += u.re * x.im + u.im * x.re;
            }
            const Cx<T> d = dinv[i];
            Xs[i][c] = Cx<T>{-(sr * d.re - si * d.im), -(sr * d.im + si * d.re)};
        }
    }
    __syncthreads();
    for (int idx = tid; idx < NB * NB; idx += 512) Uinv[idx] = Xs[idx / NB][idx % NB];
}

// Left-looking panel factorisation with the active rows in registers.
// 512 threads; thread t owns panel rows i = t + 512 r (r < R), so the panel
// height m = n - kb must be at most 512 R.  The 64 columns are processed in
// chunks of BW (8 while R <= 4, else 4: registers): (1) the U rows of the
// chunk (rows < j0) by forward substitution with the unit-lower L above it,
// one wave per column, lane = row, each x_k broadcast from its lane once
// final (the rows of L join an LDS copy as they become final); (2) the
// chunk's rows >= j0 loaded into registers and updated with
// L[:, 0:j0] U[0:j0, chunk] (left-looking: the panel's L part is read once
// per chunk instead of being rewritten after every column); (3) the chunk
// factorised column by column in registers (pivot = largest |re| + |im|,
// ties to the lowest row), its row exchanges composed and applied to the
// other panel columns in memory once per chunk; (4) written back.  At the
// end one wave composes all 64 exchanges into a (destination, source) list
// and the inverses of the 64x64 unit-lower L11 and upper U11 are formed in
// registers, eight columns per wave, lane = row.
constexpr int GF_NT = 512;

__device__ inline double rlane(double v, int k) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, k), hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline float rlane(float v, int k) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k)); }
__device__ inline int rlane(int v, int k) { return __builtin_amdgcn_readlane(v, k); }

// Composes the row exchanges (j, lp[j]), j in [jb, je), applied in order, into
// (destination, source) pairs: after them, row dst holds what was row src.
// Run by one whole wave; lane t keeps pair t in (rA, cA) and pair t + 64 in
// (rB, cB).  Returns the number of pairs.
__device__ inline int compose_swaps(const int *lp, int jb, int je, int lane, int &rA, int &cA, int &rB, int &cB) {
    rA = cA = rB = cB = -1;
    int nt = 0;
    auto find = [&](int r) -> int {
        const unsigned long long ma = __ballot(rA == r), mb = __ballot(rB == r);
        if (ma) return __ffsll((long long)ma) - 1;
        if (mb) return 64 + __ffsll((long long)mb) - 1;
        return -1;
    };
    auto put = [&](int t, int r, int c) {
        if (lane == (t & 63)) {
            if (t < 64) {
                rA = r;
                cA = c;
            } else {
                rB = r;
                cB = c;
            }
        }
    };
    for (int j = jb; j < je; ++j) {
        const int r1 = j, r2 = lp[j];
        if (r1 == r2) continue;
        int i1 = find(r1);
        if (i1 < 0) {
            i1 = nt++;
            put(i1, r1, r1);
        }
        int i2 = find(r2);
        if (i2 < 0) {
            i2 = nt++;
            put(i2, r2, r2);
        }
        const int c1 = rlane(i1 < 64 ? cA : cB, i1 & 63), c2 = rlane(i2 < 64 ? cA : cB, i2 & 63);
        put(i1, r1, c2);
        put(i2, r2, c1);
    }
    return nt;
}

// GC, GI: the element types the pointers are declared with (global address
// space for pointers read from a descriptor, so that they are not accessed as
// flat memory).
template <typename T, int R, int BW, typename GC = Cx<T>, typename GI = int32_t>
__device__ __forceinline__ void getf2r_body(int n, int kb, int w, GC *A, int64_t sA, GI *ipiv, GC *Linv, GC *Uinv,
                                            int nblk, GI *swp, GI *info, const int b) {
    constexpr int NW = GF_NT / 64;
    static_assert(BW <= NW && NB % BW == 0, "one wave per substituted column");
    __shared__ Cx<T> Ts[NB][NB + 1];  // the panel's top rows as they become final (padded: column reads)
    __shared__ Cx<T> Ux[NB][BW];
    __shared__ Cx<T> prow[BW];
    __shared__ Cx<T> xch[2][BW];
    __shared__ T red_v[NW];
    __shared__ int red_i[NW];
    __shared__ int lpiv[NB];
    __shared__ int piv_s, zero_s, nsw_s;
    __shared__ int sw_dst[2 * BW], sw_src[2 * BW];
    __shared__ Cx<T> dinv[NB];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    A += (int64_t)b * sA;
    ipiv += (int64_t)b * n;
    swp += (int64_t)b * SWP;
    Linv += ((int64_t)b * nblk + kb / NB) * NB * NB;
    Uinv += ((int64_t)b * nblk + kb / NB) * NB * NB;
    const int m = n - kb;
    GC *P = A + (int64_t)kb * n + kb;  // panel origin, row stride n
    const Cx<T> zero{T(0), T(0)};

    for (int j0 = 0; j0 < w; j0 += BW) {
        const int bw = min(BW, w - j0);
        // (1) U rows of the chunk: x_i = a_i - sum_{k<i} L_ik x_k for i < j0.  Rows
        // [j0 - BW, j0) became final in the previous chunk and join the staged
        // corner; lane i keeps a_i, and x_k is broadcast from lane k once final.
        if (j0 > 0) {
            const int r0 = j0 - BW, nT = BW * j0, nU = j0 * bw;
            for (int idx = tid; idx < nT + nU; idx += GF_NT) {
                if (idx < nT) {
                    const int i = r0 + idx / j0, k = idx % j0;
                    Ts[i][k] = P[(int64_t)i * n + k];
                } else {
                    const int q = idx - nT, i = q / bw, c = q % bw;
                    Ux[i][c] = P[(int64_t)i * n + j0 + c];
                }
            }
            __syncthreads();
            if (wave < bw) {
                const int c = wave;
                Cx<T> x = lane < j0 ? Ux[lane][c] : zero;
#pragma unroll 4
                for (int k = 0; k < j0 - 1; ++k) {
                    const Cx<T> l = (lane > k && lane < j0) ? Ts[lane][k] : zero;
                    const Cx<T> xk{rlane(x.re, k), rlane(x.im, k)};
                    x.re -= l.re * xk.re - l.im * xk.im;
                    x.im -= l.re * xk.im + l.im * xk.re;
                }
                if (lane < j0) {
                    Ux[lane][c] = x;
                    P[(int64_t)lane * n + j0 + c] = x;
                }
            }
            __syncthreads();
        }
        // (2) rows >= j0 of the chunk into registers, left-looking update
        Cx<T> a[R][BW];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = tid + GF_NT * r;
#pragma unroll
            for (int c = 0; c < BW; ++c) a[r][c] = zero;
            if (i >= j0 && i < m) {
                const GC *row = P + (int64_t)i * n;
#pragma unroll
                for (int c = 0; c < BW; ++c)
                    if (c < bw) a[r][c] = row[j0 + c];
                for (int k = 0; k < j0; ++k) {
                    const Cx<T> l = row[k];
#pragma unroll
                    for (int c = 0; c < BW; ++c) {
                        const Cx<T> u = Ux[k][c];
                        a[r][c].re -= l.re * u.re - l.im * u.im;
                        a[r][c].im -= l.re * u.im + l.im * u.re;
                    }
                }
            }
        }
        // (3) factor the chunk column by column; row exchanges happen in
        // registers here and in memory (the other panel columns) once per chunk
#pragma unroll
        for (int c = 0; c < BW; ++c) {
            if (c >= bw) break;
            const int j = j0 + c;
            T best = T(-1);
            int bi = m;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = tid + GF_NT * r;
                if (i >= j && i < m) {
                    const T v = fabs(a[r][c].re) + fabs(a[r][c].im);
                    if (v > best) {
                        best = v;
                        bi = i;
                    }
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const T ov = __shfl_xor(best, off);
                const int oi = __shfl_xor(bi, off);
                if (ov > best || (ov == best && oi < bi)) {
                    best = ov;
                    bi = oi;
                }
            }
            if (lane == 0) {
                red_v[wave] = best;
                red_i[wave] = bi;
            }
            __syncthreads();
            if (tid == 0) {
                T bv = red_v[0];
                int bx = red_i[0];
                for (int q = 1; q < NW; ++q)
                    if (red_v[q] > bv || (red_v[q] == bv && red_i[q] < bx)) {
                        bv = red_v[q];
                        bx = red_i[q];
                    }
                if (bx >= m) bx = j;
                piv_s = bx;
                lpiv[j] = bx;
                zero_s = (bv == T(0));
                if (bv == T(0) && info[b] == 0) info[b] = kb + j + 1;
            }
            __syncthreads();
            const int piv = piv_s;
            if (piv != j) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = tid + GF_NT * r;
                    if (i == j)
#pragma unroll
                        for (int cc = 0; cc < BW; ++cc) xch[0][cc] = a[r][cc];
                    if (i == piv)
#pragma unroll
                        for (int cc = 0; cc < BW; ++cc) xch[1][cc] = a[r][cc];
                }
                __syncthreads();
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = tid + GF_NT * r;
                    if (i == j)
#pragma unroll
                        for (int cc = 0; cc < BW; ++cc) a[r][cc] = xch[1][cc];
                    if (i == piv)
#pragma unroll
                        for (int cc = 0; cc < BW; ++cc) a[r][cc] = xch[0][cc];
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (tid + GF_NT * r == j)
#pragma unroll
                    for (int cc = 0; cc < BW; ++cc) prow[cc] = a[r][cc];
            __syncthreads();
            if (!zero_s) {
                const Cx<T> inv = crcp(prow[c]);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = tid + GF_NT * r;
                    if (i > j && i < m) {
                        const Cx<T> l = cmul(a[r][c], inv);
                        a[r][c] = l;
#pragma unroll
                        for (int cc = 0; cc < BW; ++cc)
                            if (cc > c) {
                                const Cx<T> u = prow[cc];
                                a[r][cc].re -= l.re * u.re - l.im * u.im;
                                a[r][cc].im -= l.re * u.im + l.im * u.re;
                            }
                    }
                }
            }
            __syncthreads();
        }
        // the chunk's exchanges, composed, on the panel columns outside it
        if (wave == 0) {
            int rA, cA, rB, cB;
            const int nt = compose_swaps(lpiv, j0, j0 + bw, lane, rA, cA, rB, cB);
            if (lane < nt) {
                sw_dst[lane] = rA;
                sw_src[lane] = cA;
            }
            if (lane == 0) nsw_s = nt;
        }
        __syncthreads();
        {
            const int nt = nsw_s, oc = w - bw;  // columns [0, j0) and [j0 + bw, w)
            constexpr int MAXP = (2 * BW * NB + GF_NT - 1) / GF_NT;
            Cx<T> v[MAXP];
#pragma unroll
            for (int q = 0; q < MAXP; ++q) {
                const int idx = tid + GF_NT * q;
                if (idx < nt * oc) {
                    const int t = idx / oc, cc = idx % oc, col = cc < j0 ? cc : cc + bw;
                    v[q] = P[(int64_t)sw_src[t] * n + col];
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < MAXP; ++q) {
                const int idx = tid + GF_NT * q;
                if (idx < nt * oc) {
                    const int t = idx / oc, cc = idx % oc, col = cc < j0 ? cc : cc + bw;
                    P[(int64_t)sw_dst[t] * n + col] = v[q];
                }
            }
        }
        // (4) the chunk back to memory
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = tid + GF_NT * r;
            if (i >= j0 && i < m)
#pragma unroll
                for (int c = 0; c < BW; ++c)
                    if (c < bw) P[(int64_t)i * n + j0 + c] = a[r][c];
        }
        __syncthreads();
    }

    if (tid < w) ipiv[kb + tid] = kb + lpiv[tid];
    // all of the panel's exchanges as one (destination, source) list
    if (wave == 0) {
        int rA, cA, rB, cB;
        const int nt = compose_swaps(lpiv, 0, w, lane, rA, cA, rB, cB);
        if (lane == 0) swp[0] = nt;
        if (lane < nt) {
            swp[1 + lane] = kb + rA;
            swp[1 + 2 * NB + lane] = kb + cA;
        }
        if (lane + 64 < nt) {
            swp[1 + 64 + lane] = kb + rB;
            swp[1 + 2 * NB + 64 + lane] = kb + cB;
        }
    }
    // the factored 64 x 64 corner, zero padded, and the inverses of its unit
    // lower and upper triangles, eight columns per wave with lane = row
    for (int idx = tid; idx < NB * NB; idx += GF_NT) {
        const int i = idx / NB, c = idx % NB;
        Ts[i][c] = (i < w && c < w) ? P[(int64_t)i * n + c] : zero;
    }
    __syncthreads();
    if (tid < w) dinv[tid] = crcp(Ts[tid][tid]);
    __syncthreads();
    constexpr int CPW = NB / NW;
    Cx<T> x[CPW];
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
        const int c = wave * CPW + q;
        x[q] = (lane == c && c < w) ? Cx<T>{T(1), T(0)} : zero;
    }
    for (int k = 0; k < w - 1; ++k) {
        const Cx<T> l = (lane > k && lane < w) ? Ts[lane][k] : zero;
#pragma unroll
        for (int q = 0; q < CPW; ++q) {
            const Cx<T> xk{rlane(x[q].re, k), rlane(x[q].im, k)};
            x[q].re -= l.re * xk.re - l.im * xk.im;
            x[q].im -= l.re * xk.im + l.im * xk.re;
        }
    }
#pragma unroll
    for (int q = 0; q < CPW; ++q) Linv[lane * NB + wave * CPW + q] = x[q];
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
        const int c = wave * CPW + q;
        x[q] = (lane == c && c < w) ? Cx<T>{T(1), T(0)} : zero;
    }
    for (int k = w - 1; k >= 0; --k) {
        const Cx<T> d = dinv[k];
        const Cx<T> u = lane < k ? Ts[lane][k] : zero;
#pragma unroll
        for (int q = 0; q < CPW; ++q) {
            if (lane == k) x[q] = cmul(x[q], d);
            const Cx<T> xk{rlane(x[q].re, k), rlane(x[q].im, k)};
            x[q].re -= u.re * xk.re - u.im * xk.im;
            x[q].im -= u.re * xk.im + u.im * xk.re;
        }
    }
#pragma unroll
    for (int q = 0; q < CPW; ++q) Uinv[lane * NB + wave * CPW + q] = x[q];
}

template <typename T, int R, int BW>
__global__ __launch_bounds__(GF_NT) void k_getf2r(int n, int kb, int w, Cx<T> *A, int64_t sA, int32_t *ipiv,
                                                  Cx<T> *Linv, Cx<T> *Uinv, int nblk, int32_t *swp, int32_t *info) {
    getf2r_body<T, R, BW>(n, kb, w, A, sA, ipiv, Linv, Uinv, nblk, swp, info, blockIdx.x);
}

// The index of the item whose workgroups wg0 .. include g (items ordered by wg0).
__device__ inline int group_item(const PanelItem *__restrict__ it, int n_items, int64_t g) {
    int a = 0, b = n_items - 1;
    while (a < b) {
        const int m = (a + b + 1) >> 1;
        if (it[m].wg0 <= g) a = m;
        else b = m - 1;
    }
    return a;
}

// Many batched panel factorisations in one launch (the batched driver's lock
// steps): workgroup g factorises batch entry g - wg0 of its item.
template <typename T, int R, int BW>
__global__ __launch_bounds__(GF_NT) void k_getf2r_group(const PanelItem *__restrict__ items, int n_items) {
    const PanelItem p = items[group_item(items, n_items, blockIdx.x)];
    typedef dglobal<Cx<T>> GC;
    typedef dglobal<int32_t> GI;
    getf2r_body<T, R, BW, GC, GI>(p.n, p.kb, p.w, (GC *)p.A, p.sA, (GI *)p.ipiv, (GC *)p.Linv, (GC *)p.Uinv, p.nblk,
                                  (GI *)p.swp, (GI *)p.info, (int)(blockIdx.x - p.wg0));
}

// Apply a panel's composed row exchanges to columns [0, kb) and [kb+w, n).
// Workgroup = 32 columns, eight threads per column, each holding up to 16 of
// the (at most 2 NB) source values in registers: all loads are issued before
// any store, and every source row is read before any row is written (one
// barrier).  No LDS, so the pass runs at full occupancy.
template <typename T, typename GC = Cx<T>, typename GI = const int32_t>
__device__ __forceinline__ void laswp_body(int n, int kb, int w, GC *A, int64_t sA, GI *swp, const int b,
                                           const int cg) {
    constexpr int PER = 2 * NB / 8;
    A += (int64_t)b * sA;
    swp += (int64_t)b * SWP;
    const int nt = swp[0];
    if (nt == 0) return;
    const int ncols = n - w;
    const int cc = threadIdx.x & 31, tr = threadIdx.x >> 5;
    const int idx = cg * 32 + cc;
    const int c = idx < kb ? idx : idx + w;
    const bool ok = idx < ncols;
    T vr[PER], vi[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int t = tr + 8 * q;
        vr[q] = vi[q] = T(0);
        if (ok && t < nt) {
            const GC &x = A[(int64_t)swp[1 + 2 * NB + t] * n + c];
            vr[q] = x.re;
            vi[q] = x.im;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int t = tr + 8 * q;
        if (ok && t < nt) {
            GC &x = A[(int64_t)swp[1 + t] * n + c];
            x.re = vr[q];
            x.im = vi[q];
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_laswp(int n, int kb, int w, Cx<T> *A, int64_t sA, const int32_t *swp) {
    laswp_body<T>(n, kb, w, A, sA, swp, blockIdx.y, blockIdx.x);
}

// Many batched row-exchange passes in one launch: an item's workgroups are
// (batch entry, 32-column group) pairs, column groups fastest.
template <typename T>
__global__ __launch_bounds__(256) void k_laswp_group(const PanelItem *__restrict__ items, int n_items) {
    const PanelItem p = items[group_item(items, n_items, blockIdx.x)];
    const int ncg = (p.n - p.w + 31) / 32;
    const int64_t r = blockIdx.x - p.wg0;
    typedef dglobal<Cx<T>> GC;
    typedef dglobal<const int32_t> GI;
    laswp_body<T, GC, GI>(p.n, p.kb, p.w, (GC *)p.A, p.sA, (GI *)p.swp, (int)(r / ncg), (int)(r % ncg));
}

// Full row permutation of a factorisation: row i of P A is row perm[i] of A.
__global__ __launch_bounds__(256) void k_perm_from_ipiv(int n, const int32_t *ipiv, int32_t *perm) {
    extern __shared__ int32_t pm[];
    const int b = blockIdx.x;
    ipiv += (int64_t)b * n;
    perm += (int64_t)b * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) pm[i] = i;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int j = 0; j < n; ++j) {
            const int r = ipiv[j];
            if (r != j) {
                const int t = pm[j];
                pm[j] = pm[r];
                pm[r] = t;
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) perm[i] = pm[i];
}

// B[b][i][c] = src[b][perm[i]][c]  (out of place gather of rows)
// Grid of the row-wise copies below: x = 256-column blocks, y = rows and
// z = batch entries, each walked with its grid stride (no division per
// element).  About 64k workgroups in all, so that each copies many rows
// (one 4-KB row segment per workgroup left the copies at 3.7 TB/s, bound by
// launching workgroups).
inline dim3 rows_grid(int rows, int cols, int batch) {
    const int xb = (cols + 255) / 256, zb = std::min(batch, 65535);
    const int yb = std::max(1, std::min(rows, 65536 / std::max(1, xb * zb)));
    return dim3((unsigned)xb, (unsigned)yb, (unsigned)zb);
}

template <typename T>
__global__ void k_rowgather(int n, int nrhs, int batch, const int32_t *perm, const Cx<T> *src, int64_t sS,
                            Cx<T> *dst, int64_t sD) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nrhs) return;
    for (int b = blockIdx.z; b < batch; b += gridDim.z)
        for (int i = blockIdx.y; i < n; i += gridDim.y)
            dst[(int64_t)b * sD + (int64_t)i * nrhs + c] =
                src[(int64_t)b * sS + (int64_t)perm[(int64_t)b * n + i] * nrhs + c];
}

// B[b][i][c] = v[perm[i]][c] (dense real v) or delta(perm[i], c) lam[c] (diagonal);
// perm may be null (identity).
__global__ void k_init_rhs(int n, int batch, const double *v, int v_is_diag, const int32_t *perm, zdbl *B,
                           int64_t sB) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    for (int b = blockIdx.z; b < batch; b += gridDim.z)
        for (int i = blockIdx.y; i < n; i += gridDim.y) {
            const int r = perm ? perm[(int64_t)b * n + i] : i;
            double x;
            if (v_is_diag) x = (r == c) ? v[c] : 0.0;
            else x = v[(int64_t)r * n + c];
            B[(int64_t)b * sB + (int64_t)i * n + c] = zdbl{x, 0.0};
        }
}

__global__ void k_conj_mirror(int64_t nn, int n_omega, zdbl *W) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + blockIdx.y;  // 1 .. n_omega/2 - 1
    if (idx >= nn) return;
    const zdbl s = W[(int64_t)(n_omega - j) * nn + idx];
    W[(int64_t)j * nn + idx] = zdbl{s.re, -s.im};
}

__global__ void k_z2c(const zdbl *src, zflt *dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = zflt{(float)src[i].re, (float)src[i].im};
}

// W[b] += d[b] for active batch entries (d complex float).
__global__ void k_c2z_add(const zflt *d, zdbl *W, int64_t n_per, const int32_t *active) {
    const int b = blockIdx.y;
    if (active && !active[b]) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_per; i += (int64_t)gridDim.x * blockDim.x) {
        const zflt x = d[(int64_t)b * n_per + i];
        zdbl &y = W[(int64_t)b * n_per + i];
        y.re += (double)x.re;
        y.im += (double)x.im;
    }
}

// out[2b] += sum |d|^2, out[2b+1] += sum |W|^2 (caller zeroes out).
__global__ void k_norms(const zflt *d, const zdbl *W, int64_t n_per, double *out) {
    const int b = blockIdx.y;
    double sd = 0, sw = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_per; i += (int64_t)gridDim.x * blockDim.x) {
        const zflt x = d[(int64_t)b * n_per + i];
        const zdbl y = W[(int64_t)b * n_per + i];
        sd += (double)x.re * x.re + (double)x.im * x.im;
        sw += y.re * y.re + y.im * y.im;
    }
    for (int off = 32; off > 0; off >>= 1) {
        sd += __shfl_xor(sd, off);
        sw += __shfl_xor(sw, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&out[2 * b], sd);
        atomicAdd(&out[2 * b + 1], sw);
    }
}


__global__ void k_rowgather_z2c(int n, int nrhs, int batch, const int32_t *perm, const zdbl *src, int64_t sS,
                                zflt *dst, int64_t sD) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nrhs) return;
    for (int b = blockIdx.z; b < batch; b += gridDim.z)
        for (int i = blockIdx.y; i < n; i += gridDim.y) {
            const zdbl x = src[(int64_t)b * sS + (int64_t)perm[(int64_t)b * n + i] * nrhs + c];
            dst[(int64_t)b * sD + (int64_t)i * nrhs + c] = zflt{(float)x.re, (float)x.im};
        }
}

__global__ void k_c2z_set(const zflt *d, zdbl *W, int64_t n_per) {
    const int b = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_per; i += (int64_t)gridDim.x * blockDim.x) {
        const zflt x = d[(int64_t)b * n_per + i];
        W[(int64_t)b * n_per + i] = zdbl{(double)x.re, (double)x.im};
    }
}

// dst[c][r] = src[r][c] through a 32x32 LDS tile
__global__ __launch_bounds__(256) void k_transpose_d(int rows, int cols, const double *src, double *dst) {
    __shared__ double t[32][33];
    const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = ty; k < 32; k += 8)
        if (r0 + k < rows && c0 + tx < cols) t[k][tx] = src[(int64_t)(r0 + k) * cols + c0 + tx];
    __syncthreads();
    for (int k = ty; k < 32; k += 8)
        if (c0 + k < cols && r0 + tx < rows) dst[(int64_t)(c0 + k) * rows + r0 + tx] = t[tx][k];
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
hipError_t gemm_t(hipStream_t st, int M, int N, int K, T alpha, const Cx<T> *A, int64_t lda, int64_t sA,
                  const Cx<T> *B, int64_t ldb, int64_t sB, T beta, Cx<T> *C, int64_t ldc, int64_t sC, int batch);
template <>
hipError_t gemm_t<double>(hipStream_t st, int M, int N, int K, double alpha, const Cx<double> *A, int64_t lda,
                          int64_t sA, const Cx<double> *B, int64_t ldb, int64_t sB, double beta, Cx<double> *C,
                          int64_t ldc, int64_t sC, int batch) {
    return launch_zgemm_lu(st, M, N, K, alpha, (const zdbl *)A, lda, sA, (const zdbl *)B, ldb, sB, beta, (zdbl *)C,
                           ldc, sC, batch);
}
template <>
hipError_t gemm_t<float>(hipStream_t st, int M, int N, int K, float alpha, const Cx<float> *A, int64_t lda,
                         int64_t sA, const Cx<float> *B, int64_t ldb, int64_t sB, float beta, Cx<float> *C,
                         int64_t ldc, int64_t sC, int batch) {
    return launch_cgemm(st, M, N, K, alpha, (const zflt *)A, lda, sA, (const zflt *)B, ldb, sB, beta, (zflt *)C, ldc,
                        sC, batch);
}

// Two-level blocking: 64-wide panels inside 256-wide blocks.  Inside a block
// each panel updates only the block's remaining columns (narrow GEMMs); the
// block then computes its U12 rows and updates the trailing matrix with one
// rank-256 GEMM, so the large updates stream the trailing matrix a quarter as
// often as rank-64 updates would.  Row exchanges of every panel are applied at
// once to all columns outside the panel (the columns right of the block have
// received no update from this block yet, so the order is the same as
// applying them all before the block's triangular solve).
constexpr int NBO = 256;

template <typename T>
hipError_t getrf_impl(hipStream_t st, int n, Cx<T> *A, int64_t sA, int32_t *ipiv, Cx<T> *Linv, Cx<T> *Uinv,
                      Cx<T> *scratch, int32_t *info, int batch) {
    const int nblk = (n + NB - 1) / NB;
    const int64_t sI = (int64_t)nblk * NB * NB;
    int32_t *swp = (int32_t *)(scratch + (int64_t)batch * NB * n);
    hipError_t e;
    OpRecorder *rec = g_rec;
    if (rec) rec->mark();
    for (int KB = 0; KB < n; KB += NBO) {
        const int WO = min(NBO, n - KB);
        for (int kb = KB; kb < KB + WO; kb += NB) {
            const int w = min(NB, n - kb);
            const int m = n - kb;
            if (rec) {
                // lock-step recording: the panel (a grouped launch per
                // register-row variant) and its row exchanges
                RecOp o;
                o.p = PanelItem{A, sA, ipiv, swp, info, Linv, Uinv, n, kb, w, nblk, batch, 0};
                if (m <= 4096) {
                    o.kind = RecOp::PANEL;
                    o.key = (m <= 512 ? 0 : m <= 1024 ? 1 : m <= 2048 ? 2 : m <= 3072 ? 3 : 4) + (sizeof(T) == 4 ? 5 : 0);
                    rec->ops.push_back(o);
                } else {
                    rec->other([=](hipStream_t s2) {
                        hipLaunchKernelGGL(k_getf2<T>, dim3(batch), dim3(512), 0, s2, n, kb, w, A, sA, ipiv, Linv,
                                           Uinv, nblk, scratch, swp, info);
                        return hipGetLastError();
                    });
                }
                if (n - w > 0) {
                    RecOp l;
                    l.kind = RecOp::LASWP;
                    l.key = sizeof(T) == 4 ? 1 : 0;
                    l.p = o.p;
                    rec->ops.push_back(l);
                }
            } else {
            ProfScope ps(st, "lu_panel", 0.0, 2.0 * m * w * sizeof(Cx<T>) * (double)batch);
            if (m <= 512)
                hipLaunchKernelGGL((k_getf2r<T, 1, 8>), dim3(batch), dim3(GF_NT), 0, st, n, kb, w, A, sA, ipiv, Linv,
                                   Uinv, nblk, swp, info);
            else if (m <= 1024)
                hipLaunchKernelGGL((k_getf2r<T, 2, 8>), dim3(batch), dim3(GF_NT), 0, st, n, kb, w, A, sA, ipiv, Linv,
                                   Uinv, nblk, swp, info);
            else if (m <= 2048)
                hipLaunchKernelGGL((k_getf2r<T, 4, 8>), dim3(batch), dim3(GF_NT), 0, st, n, kb, w, A, sA, ipiv, Linv,
                                   Uinv, nblk, swp, info);
            else if (m <= 3072)
                hipLaunchKernelGGL((k_getf2r<T, 6, 4>), dim3(batch), dim3(GF_NT), 0, st, n, kb, w, A, sA, ipiv, Linv,
                                   Uinv, nblk, swp, info);
            else if (m <= 4096)
                hipLaunchKernelGGL((k_getf2r<T, 8, 4>), dim3(batch), dim3(GF_NT), 0, st, n, kb, w, A, sA, ipiv, Linv,
                                   Uinv, nblk, swp, info);
            else
                hipLaunchKernelGGL(k_getf2<T>, dim3(batch), dim3(512), 0, st, n, kb, w, A, sA, ipiv, Linv, Uinv, nblk,
                                   scratch, swp, info);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if (n - w > 0) {
                ProfScope pl(st, "laswp", 0.0, 2.0 * w * (n - w) * sizeof(Cx<T>) * (double)batch);
                hipLaunchKernelGGL(k_laswp<T>, dim3((n - w + 31) / 32, batch), dim3(256), 0, st, n, kb, w, A, sA, swp);
                if ((e = hipGetLastError()) != hipSuccess) return e;
            }
            }
            const int rb = KB + WO - kb - w;  // columns of this block right of the panel
            if (rb > 0) {
                const Cx<T> *Lb = Linv + (int64_t)(kb / NB) * NB * NB;
                Cx<T> *A12 = A + (int64_t)kb * n + kb + w;
                e = gemm_t<T>(st, w, rb, w, T(1), Lb, NB, sI, A12, n, sA, T(0), A12, n, sA, batch);
                if (e != hipSuccess) return e;
                if (n - kb - w > 0) {
                    e = gemm_t<T>(st, n - kb - w, rb, w, T(-1), A + (int64_t)(kb + w) * n + kb, n, sA, A12, n, sA, T(1),
                                  A + (int64_t)(kb + w) * n + kb + w, n, sA, batch);
                    if (e != hipSuccess) return e;
                }
            }
        }
        const int rest = n - KB - WO;
        if (rest > 0) {
            // U12 rows of the block: blocked forward substitution over its panels
            for (int kb = KB; kb < KB + WO; kb += NB) {
                const int w = min(NB, n - kb);
                Cx<T> *Ak = A + (int64_t)kb * n + KB + WO;
                e = gemm_t<T>(st, w, rest, w, T(1), Linv + (int64_t)(kb / NB) * NB * NB, NB, sI, Ak, n, sA, T(0), Ak,
                              n, sA, batch);
                if (e != hipSuccess) return e;
                const int r2 = KB + WO - kb - w;
                if (r2 > 0) {
                    e = gemm_t<T>(st, r2, rest, w, T(-1), A + (int64_t)(kb + w) * n + kb, n, sA, Ak, n, sA, T(1),
                                  A + (int64_t)(kb + w) * n + KB + WO, n, sA, batch);
                    if (e != hipSuccess) return e;
                }
            }
            // trailing update, rank WO
            e = gemm_t<T>(st, rest, rest, WO, T(-1), A + (int64_t)(KB + WO) * n + KB, n, sA,
                          A + (int64_t)KB * n + KB + WO, n, sA, T(1), A + (int64_t)(KB + WO) * n + KB + WO, n, sA,
                          batch);
            if (e != hipSuccess) return e;
        }
    }
    if (rec) rec->mark();
    return hipSuccess;
}

// X[b][i][j] = X[b][j][i] for j > i (32 x 32 tiles through LDS).
template <typename T>
__global__ __launch_bounds__(256) void k_mirror_lower(int n, int nt, Cx<T> *X, int64_t sX) {
    __shared__ Cx<T> t[32][33];
    int tile = blockIdx.x, bi = 0;
    while (tile >= nt - bi) {  // upper tiles (bi <= bj) row by row
        tile -= nt - bi;
        ++bi;
    }
    const int bj = bi + tile;
    Cx<T> *x = X + (int64_t)blockIdx.y * sX;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = bj * 32 + ty + 8 * q, c = bi * 32 + tx;  // lower tile (bj, bi)
        if (r < n && c < n) t[ty + 8 * q][tx] = x[(int64_t)r * n + c];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = bi * 32 + ty + 8 * q, c = bj * 32 + tx;  // upper (r, c) = lower (c, r)
        if (r < n && c < n && c > r) x[(int64_t)r * n + c] = t[tx][ty + 8 * q];
    }
}

template <typename T>
hipError_t getrs_impl(hipStream_t st, int n, int nrhs, const Cx<T> *LU, int64_t sA, const Cx<T> *Linv,
                      const Cx<T> *Uinv, Cx<T> *B, int64_t sB, int batch, bool sym_lower) {
    const int nblk = (n + NB - 1) / NB;
    const int64_t sI = (int64_t)nblk * NB * NB;
    hipError_t e;
    OpRecorder *rec = g_rec;
    if (rec) rec->mark();
    // forward: L Y = P B, left-looking over the outer blocks: block row
    // [KB, KB + WO) first takes everything already solved above it in one
    // product (inner dimension KB, long for the later blocks), then is solved
    // 64 rows at a time
    for (int KB = 0; KB < n; KB += NBO) {
        const int WO = min(NBO, n - KB);
        if (KB > 0) {
            e = gemm_t<T>(st, WO, nrhs, KB, T(-1), LU + (int64_t)KB * n, n, sA, B, nrhs, sB, T(1),
                          B + (int64_t)KB * nrhs, nrhs, sB, batch);
            if (e != hipSuccess) return e;
        }
        for (int kb = KB; kb < KB + WO; kb += NB) {
            const int w = min(NB, n - kb);
            Cx<T> *Bk = B + (int64_t)kb * nrhs;
            e = gemm_t<T>(st, w, nrhs, w, T(1), Linv + (int64_t)(kb / NB) * NB * NB, NB, sI, Bk, nrhs, sB, T(0), Bk,
                          nrhs, sB, batch);
            if (e != hipSuccess) return e;
            const int r2 = KB + WO - kb - w;
            if (r2 > 0) {
                e = gemm_t<T>(st, r2, nrhs, w, T(-1), LU + (int64_t)(kb + w) * n + kb, n, sA, Bk, nrhs, sB, T(1),
                              B + (int64_t)(kb + w) * nrhs, nrhs, sB, batch);
                if (e != hipSuccess) return e;
            }
        }
    }
    // backward: U X = Y, left-looking from the last outer block up.  With
    // sym_lower, rows [r0, r1) are only needed in columns [0, r1): every
    // product is cut to those columns, so the work follows the lower triangle
    // (a right-looking update would fill whole squares of columns).
    for (int KB = ((n - 1) / NBO) * NBO; KB >= 0; KB -= NBO) {
        const int WO = min(NBO, n - KB);
        const int below = n - KB - WO;
        if (below > 0) {
            e = gemm_t<T>(st, WO, sym_lower ? KB + WO : nrhs, below, T(-1), LU + (int64_t)KB * n + KB + WO, n, sA,
                          B + (int64_t)(KB + WO) * nrhs, nrhs, sB, T(1), B + (int64_t)KB * nrhs, nrhs, sB, batch);
            if (e != hipSuccess) return e;
        }
        for (int kb = KB + ((WO - 1) / NB) * NB; kb >= KB; kb -= NB) {
            const int w = min(NB, n - kb);
            Cx<T> *Bk = B + (int64_t)kb * nrhs;
            const int cols = sym_lower ? kb + w : nrhs;
            e = gemm_t<T>(st, w, cols, w, T(1), Uinv + (int64_t)(kb / NB) * NB * NB, NB, sI, Bk, nrhs, sB, T(0), Bk,
                          nrhs, sB, batch);
            if (e != hipSuccess) return e;
            const int r2 = kb - KB;
            if (r2 > 0) {
                e = gemm_t<T>(st, r2, sym_lower ? kb : nrhs, w, T(-1), LU + (int64_t)KB * n + kb, n, sA, Bk, nrhs, sB,
                              T(1), B + (int64_t)KB * nrhs, nrhs, sB, batch);
                if (e != hipSuccess) return e;
            }
        }
    }
    if (rec) rec->mark();
    if (sym_lower && n > 1) {
        const int nt = (n + 31) / 32;
        if (rec) {
            rec->other([=](hipStream_t s2) {
                hipLaunchKernelGGL(k_mirror_lower<T>, dim3((unsigned)(nt * (nt + 1) / 2), (unsigned)batch), dim3(256),
                                   0, s2, n, nt, B, sB);
                return hipGetLastError();
            });
            return hipSuccess;
        }
        ProfScope ps(st, "mirror_lower", 0.0, 2.0 * sizeof(Cx<T>) * (double)n * (n - 1) / 2 * batch);
        hipLaunchKernelGGL(k_mirror_lower<T>, dim3((unsigned)(nt * (nt + 1) / 2), (unsigned)batch), dim3(256), 0, st,
                           n, nt, B, sB);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace

// scratch must hold batch * 64 * n complex + batch * (1 + 4*64) int32.
template <>
hipError_t getrf_batched<zdbl>(hipStream_t st, int n, zdbl *A, int64_t sA, int32_t *ipiv, zdbl *Linv, zdbl *Uinv,
                               zdbl *scratch, int32_t *info, int batch) {
    return getrf_impl<double>(st, n, (Cx<double> *)A, sA, ipiv, (Cx<double> *)Linv, (Cx<double> *)Uinv,
                              (Cx<double> *)scratch, info, batch);
}
template <>
hipError_t getrf_batched<zflt>(hipStream_t st, int n, zflt *A, int64_t sA, int32_t *ipiv, zflt *Linv, zflt *Uinv,
                               zflt *scratch, int32_t *info, int batch) {
    return getrf_impl<float>(st, n, (Cx<float> *)A, sA, ipiv, (Cx<float> *)Linv, (Cx<float> *)Uinv,
                             (Cx<float> *)scratch, info, batch);
}
template <>
hipError_t getrs_batched<zdbl>(hipStream_t st, int n, int nrhs, const zdbl *LU, int64_t sA, const int32_t *ipiv,
                               const zdbl *Linv, const zdbl *Uinv, zdbl *B, int64_t sB, int batch, bool sym_lower) {
    (void)ipiv;  // rows of B are already in pivot order (see launch_perm / launch_init_rhs)
    return getrs_impl<double>(st, n, nrhs, (const Cx<double> *)LU, sA, (const Cx<double> *)Linv,
                              (const Cx<double> *)Uinv, (Cx<double> *)B, sB, batch, sym_lower && nrhs == n);
}
template <>
hipError_t getrs_batched<zflt>(hipStream_t st, int n, int nrhs, const zflt *LU, int64_t sA, const int32_t *ipiv,
                               const zflt *Linv, const zflt *Uinv, zflt *B, int64_t sB, int batch, bool sym_lower) {
    (void)ipiv;
    return getrs_impl<float>(st, n, nrhs, (const Cx<float> *)LU, sA, (const Cx<float> *)Linv,
                             (const Cx<float> *)Uinv, (Cx<float> *)B, sB, batch, sym_lower && nrhs == n);
}

hipError_t launch_perm(hipStream_t st, int n, const int32_t *ipiv, int32_t *perm, int batch) {
    GW_DEFER(launch_perm(st, n, ipiv, perm, batch));
    hipLaunchKernelGGL(k_perm_from_ipiv, dim3(batch), dim3(256), (size_t)n * sizeof(int32_t), st, n, ipiv, perm);
    return hipGetLastError();
}

hipError_t launch_rowgather_c(hipStream_t st, int n, int nrhs, const int32_t *perm, const zflt *src, int64_t sS,
                              zflt *dst, int64_t sD, int batch) {
    GW_DEFER(launch_rowgather_c(st, n, nrhs, perm, src, sS, dst, sD, batch));
    hipLaunchKernelGGL(k_rowgather<float>, rows_grid(n, nrhs, batch), dim3(256), 0, st, n, nrhs, batch, perm,
                       (const Cx<float> *)src, sS, (Cx<float> *)dst, sD);
    return hipGetLastError();
}
hipError_t launch_rowgather_z(hipStream_t st, int n, int nrhs, const int32_t *perm, const zdbl *src, int64_t sS,
                              zdbl *dst, int64_t sD, int batch) {
    GW_DEFER(launch_rowgather_z(st, n, nrhs, perm, src, sS, dst, sD, batch));
    hipLaunchKernelGGL(k_rowgather<double>, rows_grid(n, nrhs, batch), dim3(256), 0, st, n, nrhs, batch, perm,
                       (const Cx<double> *)src, sS, (Cx<double> *)dst, sD);
    return hipGetLastError();
}

hipError_t launch_init_rhs_perm(hipStream_t st, int n, const double *v, int v_is_diag, const int32_t *perm, zdbl *B,
                                int64_t sB, int batch) {
    GW_DEFER(launch_init_rhs_perm(st, n, v, v_is_diag, perm, B, sB, batch));
    ProfScope ps(st, "init_rhs", 0.0, 16.0 * (double)n * n * batch);
    hipLaunchKernelGGL(k_init_rhs, rows_grid(n, n, batch), dim3(256), 0, st, n, batch, v, v_is_diag, perm, B, sB);
    return hipGetLastError();
}

hipError_t launch_init_rhs(hipStream_t st, int n, const double *v, int v_is_diag, zdbl *B, int64_t sB, int batch) {
    return launch_init_rhs_perm(st, n, v, v_is_diag, nullptr, B, sB, batch);
}

hipError_t launch_conj_mirror(hipStream_t st, int64_t nn, int n_omega, zdbl *W) {
    GW_DEFER(launch_conj_mirror(st, nn, n_omega, W));
    if (n_omega < 4) return hipSuccess;
    dim3 grid((unsigned)((nn + 255) / 256), n_omega / 2 - 1);
    ProfScope ps(st, "conj_mirror", 0.0, 2.0 * 16.0 * (double)nn * (n_omega / 2 - 1));
    hipLaunchKernelGGL(k_conj_mirror, grid, dim3(256), 0, st, nn, n_omega, W);
    return hipGetLastError();
}

hipError_t launch_z2c(hipStream_t st, const zdbl *src, zflt *dst, int64_t n) {
    GW_DEFER(launch_z2c(st, src, dst, n));
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_z2c, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_c2z_add(hipStream_t st, const zflt *d, zdbl *W, int64_t n_per, int batch, const int32_t *active) {
    GW_DEFER(launch_c2z_add(st, d, W, n_per, batch, active));
    int64_t blocks = (n_per + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_c2z_add, dim3((unsigned)blocks, batch), dim3(256), 0, st, d, W, n_per, active);
    return hipGetLastError();
}

hipError_t launch_norms(hipStream_t st, const zflt *dW, const zdbl *W, int64_t n_per, int batch, double *out) {
    GW_DEFER(launch_norms(st, dW, W, n_per, batch, out));
    int64_t blocks = (n_per + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_norms, dim3((unsigned)blocks, batch), dim3(256), 0, st, dW, W, n_per, out);
    return hipGetLastError();
}

hipError_t launch_rowgather_z2c(hipStream_t st, int n, int nrhs, const int32_t *perm, const zdbl *src, int64_t sS,
                                zflt *dst, int64_t sD, int batch) {
    GW_DEFER(launch_rowgather_z2c(st, n, nrhs, perm, src, sS, dst, sD, batch));
    hipLaunchKernelGGL(k_rowgather_z2c, rows_grid(n, nrhs, batch), dim3(256), 0, st, n, nrhs, batch, perm, src, sS,
                       dst, sD);
    return hipGetLastError();
}

hipError_t launch_c2z_set(hipStream_t st, const zflt *d, zdbl *W, int64_t n_per, int batch) {
    GW_DEFER(launch_c2z_set(st, d, W, n_per, batch));
    int64_t blocks = (n_per + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_c2z_set, dim3((unsigned)blocks, batch), dim3(256), 0, st, d, W, n_per);
    return hipGetLastError();
}

// Panel keys: (R, BW) = (1, 8), (2, 8), (4, 8), (6, 4), (8, 4) for panels of at
// most 512, 1024, 2048, 3072, 4096 rows, complex double; +5 complex float.
hipError_t launch_panel_group(hipStream_t st, int key, const PanelItem *items, int n_items, int64_t n_wg) {
    if (n_items <= 0 || n_wg <= 0) return hipSuccess;
    if (key < 0 || key > 9 || n_wg > INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid((unsigned)n_wg), blk(GF_NT);
    switch (key) {
        case 0: hipLaunchKernelGGL((k_getf2r_group<double, 1, 8>), grid, blk, 0, st, items, n_items); break;
        case 1: hipLaunchKernelGGL((k_getf2r_group<double, 2, 8>), grid, blk, 0, st, items, n_items); break;
        case 2: hipLaunchKernelGGL((k_getf2r_group<double, 4, 8>), grid, blk, 0, st, items, n_items); break;
        case 3: hipLaunchKernelGGL((k_getf2r_group<double, 6, 4>), grid, blk, 0, st, items, n_items); break;
        case 4: hipLaunchKernelGGL((k_getf2r_group<double, 8, 4>), grid, blk, 0, st, items, n_items); break;
        case 5: hipLaunchKernelGGL((k_getf2r_group<float, 1, 8>), grid, blk, 0, st, items, n_items); break;
        case 6: hipLaunchKernelGGL((k_getf2r_group<float, 2, 8>), grid, blk, 0, st, items, n_items); break;
        case 7: hipLaunchKernelGGL((k_getf2r_group<float, 4, 8>), grid, blk, 0, st, items, n_items); break;
        case 8: hipLaunchKernelGGL((k_getf2r_group<float, 6, 4>), grid, blk, 0, st, items, n_items); break;
        default: hipLaunchKernelGGL((k_getf2r_group<float, 8, 4>), grid, blk, 0, st, items, n_items); break;
    }
    return hipGetLastError();
}

// Row-exchange keys: 0 complex double, 1 complex float.
hipError_t launch_laswp_group(hipStream_t st, int key, const PanelItem *items, int n_items, int64_t n_wg) {
    if (n_items <= 0 || n_wg <= 0) return hipSuccess;
    if (key < 0 || key > 1 || n_wg > INT32_MAX) return hipErrorInvalidValue;
    if (key == 0) hipLaunchKernelGGL(k_laswp_group<double>, dim3((unsigned)n_wg), dim3(256), 0, st, items, n_items);
    else hipLaunchKernelGGL(k_laswp_group<float>, dim3((unsigned)n_wg), dim3(256), 0, st, items, n_items);
    return hipGetLastError();
}

hipError_t launch_copy(hipStream_t st, void *dst, const void *src, size_t bytes) {
    GW_DEFER(launch_copy(st, dst, src, bytes));
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
}

hipError_t launch_transpose_d(hipStream_t st, int rows, int cols, const double *src, double *dst) {
    dim3 grid((cols + 31) / 32, (rows + 31) / 32);
    hipLaunchKernelGGL(k_transpose_d, grid, dim3(256), 0, st, rows, cols, src, dst);
    return hipGetLastError();
}

hipError_t launch_fill_u32(hipStream_t st, uint32_t *p, int64_t n, uint32_t value) {
    GW_DEFER(launch_fill_u32(st, p, n, value));
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, value);
    return hipGetLastError();
}

}  // namespace gwk
