// Dense products on the CDNA4 matrix cores (MFMA), for the W solve:
// forming A = 1 - v chi0, the trailing updates of the blocked LU, the
// triangular block products of the solve, and the FP64 refinement residual
// (Section 2 eq. Coulombscreening, Section 3 eq. tensorform-scr-inter).
//
// Complex numbers are interleaved {re, im}.  The products of the FP64 LU and
// solves use three real MFMA products per complex product, ac, bd and
// (a + b)(c + d) (a quarter less matrix-core work, normwise as accurate); the
// FP64 refinement residual and the FP32 products use four.
// Tiles: 256-thread workgroups, four 64-wide waves in 2x2.  An FP64 MFMA
// 16x16x4 occupies the matrix pipe for many cycles, so the complex FP64
// products are latency-bound by the LDS and global loads around it unless
// several workgroups share a CU: they use narrow tiles, 64x32 (each wave 2x1
// MFMA 16x16 blocks) at five waves per SIMD in the three-product form (94
// registers) for every LU and solve product, and 128x32 (4x1) at four waves
// per SIMD in the four-product form.  The real-times-complex and FP32
// products keep 64x64 (K steps of 16) and 128x64 (K steps of 8) at two waves
// per SIMD.  The narrow tiles are dealt to the XCDs in contiguous ranges (each
// XCD has its own L2).  K is staged through a double-buffered LDS tile, the
// next step prefetched into registers.
#include "gw_internal.h"
#include "gw_prof.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace gwk {

namespace {

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 op(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // result element e of lane l is D[(l / 16) + 4 e][l % 16] (measured on gfx950)
    static __device__ inline int row(int lane, int e) { return (lane >> 4) + 4 * e; }
};
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 op(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // result element e of lane l is D[4 (l / 16) + e][l % 16]
    static __device__ inline int row(int lane, int e) { return 4 * (lane >> 4) + e; }
};

// C = alpha * A * B + beta * C (+ identity on the real diagonal if add_eye).
// AC/BC: A/B complex (else real).  C is complex unless both are real.
// Optional C32: a complex-float copy of the result (same ld).
// Workgroup = 256 threads = 2x2 waves; a wave owns WM x WN MFMA blocks of
// 16x16, so the workgroup tile is (32 WM) x (32 WN); K advances BK per
// LDS stage.
// M3 (complex times complex only): three real products per complex product,
// (a + ib)(c + id) = ac - bd + i[(a + b)(c + d) - ac - bd], instead of four:
// a quarter fewer matrix-core operations, with the sums a + b and c + d
// formed from the operands as they come out of LDS.  Normwise as accurate
// (the imaginary part of an entry loses relative accuracy only where it is
// small against |a||c| + |b||d|); the LU and the solves use it, the FP64
// refinement residual does not.
// One (32 WM) x (32 WN) tile of C with its top-left corner at (m0, n0); A, B,
// C (and C32) point at the tile's batch entry.
// MIR: row r >= 1 of C is also written, conjugated, r rows before C's first
// row (C(-omega) = C(omega)* for a C whose rows are omega_r on a symmetric
// mesh starting at omega = 0).
template <typename T, bool AC, bool BC, int WM, int WN, int BK, bool M3, typename GT = T, bool MIR = false>
__device__ __forceinline__ void gemm_tile(int M, int N, int K, T alpha, const GT *__restrict__ A, int64_t lda,
                                          const GT *B, int64_t ldb, T beta, GT *C, int64_t ldc, int add_eye,
                                          float *C32, int m0, int n0) {
    static_assert(!M3 || (AC && BC), "the three-product form is for complex times complex");
    constexpr int BM = 32 * WM, BN = 32 * WN;
    constexpr bool CC = AC || BC;
    constexpr int ea = AC ? 2 : 1, eb = BC ? 2 : 1, ec = CC ? 2 : 1;
    constexpr int EA = BM * BK / 256, TPRA = BK / EA;  // elements per thread, threads per row (A)
    constexpr int EB = BK * BN / 256, TPRB = BN / EB;  // (B)
    static_assert(EA >= 1 && EB >= 1 && TPRA >= 1 && TPRB >= 1, "tile too small");
    typedef typename Mfma<T>::v4 v4;
    // in the three-product tile and the Cauchy product's (MIR) the
    // transposed A rows are padded by one value: unpadded, the K rows of the
    // tile are a multiple of the LDS bank span apart, so the stores of a wave
    // (several K rows of few tile rows) pile onto the same banks (3x the
    // bank-conflict cycles at 64x32; the Cauchy product reads 10% more and
    // runs 3% slower unpadded).  The other tiles run faster unpadded (the
    // four-product 128x32 of the FP64 refinement residual lost 9% to the
    // padding).  The 64x64 tile also gives each thread B columns TPRB apart.
    constexpr int PA = (M3 || MIR) ? 1 : 0;
    constexpr int SB = (BK == 16) ? TPRB : 1;
    // complex operands are staged interleaved {re, im}: one 16-byte LDS read
    // per operand value instead of two 8-byte ones
    typedef T T2 __attribute__((ext_vector_type(2)));
    __shared__ T Ar[2][AC ? 1 : BK][AC ? 1 : BM + PA];
    __shared__ T2 Ac[2][AC ? BK : 1][AC ? BM + PA : 1];
    __shared__ T Br[2][BC ? 1 : BK][BC ? 1 : BN];
    __shared__ T2 Bc[2][BC ? BK : 1][BC ? BN : 1];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    // M3: accr = sum a c, acci = sum b d, accs = sum (a + b)(c + d)
    v4 accr[WM][WN], acci[WM][WN], accs[M3 ? WM : 1][M3 ? WN : 1];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            accr[i][j] = v4{0, 0, 0, 0};
            acci[i][j] = v4{0, 0, 0, 0};
            if constexpr (M3) accs[i][j] = v4{0, 0, 0, 0};
        }

    const int a_row = tid / TPRA, a_k = (tid % TPRA) * EA;
    const int b_row = tid / TPRB, b_col = (SB == 1) ? (tid % TPRB) * EB : tid % TPRB;
    T ra_r[EA], ra_i[EA], rb_r[EB], rb_i[EB];
    // interior tiles take an unpredicated path
    const bool rows_in = m0 + BM <= M;
    const bool cols_in = n0 + BN <= N;
    auto gload = [&](int k0) {
        const int gr = m0 + a_row;
        if (rows_in && k0 + BK <= K) {
            const GT *p = A + ((int64_t)gr * lda + k0 + a_k) * ea;
#pragma unroll
            for (int c = 0; c < EA; ++c) {
                ra_r[c] = p[c * ea];
                if constexpr (AC) ra_i[c] = p[c * ea + 1];
                else ra_i[c] = T(0);
            }
        } else {
#pragma unroll
            for (int c = 0; c < EA; ++c) {
                const int gk = k0 + a_k + c;
                if (gr < M && gk < K) {
                    const GT *p = A + ((int64_t)gr * lda + gk) * ea;
                    ra_r[c] = p[0];
                    if constexpr (AC) ra_i[c] = p[1];
                    else ra_i[c] = T(0);
                } else {
                    ra_r[c] = T(0);
                    ra_i[c] = T(0);
                }
            }
        }
        const int gk = k0 + b_row;
        if (cols_in && gk < K) {
            const GT *p = B + ((int64_t)gk * ldb + n0 + b_col) * eb;
#pragma unroll
            for (int c = 0; c < EB; ++c) {
                rb_r[c] = p[c * SB * eb];
                if constexpr (BC) rb_i[c] = p[c * SB * eb + 1];
                else rb_i[c] = T(0);
            }
        } else {
#pragma unroll
            for (int c = 0; c < EB; ++c) {
                const int gc = n0 + b_col + c * SB;
                if (gk < K && gc < N) {
                    const GT *p = B + ((int64_t)gk * ldb + gc) * eb;
                    rb_r[c] = p[0];
                    if constexpr (BC) rb_i[c] = p[1];
                    else rb_i[c] = T(0);
                } else {
                    rb_r[c] = T(0);
                    rb_i[c] = T(0);
                }
            }
        }
    };
    auto lstore = [&](int b) {
#pragma unroll
        for (int c = 0; c < EA; ++c) {
            if constexpr (AC) Ac[b][a_k + c][a_row] = T2{ra_r[c], ra_i[c]};
            else Ar[b][a_k + c][a_row] = ra_r[c];
        }
#pragma unroll
        for (int c = 0; c < EB; ++c) {
            if constexpr (BC) Bc[b][b_row][b_col + c * SB] = T2{rb_r[c], rb_i[c]};
            else Br[b][b_row][b_col + c * SB] = rb_r[c];
        }
    };
    // LDS double buffer: compute on one buffer while the next K step is
    // written into the other; one barrier per K step.
    gload(0);
    lstore(0);
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < K; k0 += BK) {
        const bool more = k0 + BK < K;
        if (more) gload(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int kl = kk + (lane >> 4);
            T ar[WM], ai[WM], br[WN], bi[WN];
#pragma unroll
            for (int i = 0; i < WM; ++i) {
                const int r = wm * 16 * WM + i * 16 + (lane & 15);
                if constexpr (AC) {
                    const T2 a2 = Ac[cur][kl][r];
                    ar[i] = a2.x;
                    ai[i] = a2.y;
                } else {
                    ar[i] = Ar[cur][kl][r];
                    ai[i] = T(0);
                }
            }
#pragma unroll
            for (int j = 0; j < WN; ++j) {
                const int c = wn * 16 * WN + j * 16 + (lane & 15);
                if constexpr (BC) {
                    const T2 b2 = Bc[cur][kl][c];
                    br[j] = b2.x;
                    bi[j] = b2.y;
                } else {
                    br[j] = Br[cur][kl][c];
                    bi[j] = T(0);
                }
            }
            if constexpr (M3) {
                // three passes, each over every block, so that no MFMA waits
                // on the one issued just before it
                T sa[WM], sb[WN];
#pragma unroll
                for (int i = 0; i < WM; ++i) sa[i] = ar[i] + ai[i];
#pragma unroll
                for (int j = 0; j < WN; ++j) sb[j] = br[j] + bi[j];
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < WN; ++j) accr[i][j] = Mfma<T>::op(ar[i], br[j], accr[i][j]);
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < WN; ++j) acci[i][j] = Mfma<T>::op(ai[i], bi[j], acci[i][j]);
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < WN; ++j) accs[i][j] = Mfma<T>::op(sa[i], sb[j], accs[i][j]);
                continue;
            }
            // two passes so that no MFMA waits on the one issued just before it
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j) {
                    accr[i][j] = Mfma<T>::op(ar[i], br[j], accr[i][j]);
                    if constexpr (BC) acci[i][j] = Mfma<T>::op(ar[i], bi[j], acci[i][j]);
                    else if constexpr (AC) acci[i][j] = Mfma<T>::op(ai[i], br[j], acci[i][j]);
                }
            if constexpr (AC && BC) {
#pragma unroll
                for (int i = 0; i < WM; ++i)
#pragma unroll
                    for (int j = 0; j < WN; ++j) {
                        accr[i][j] = Mfma<T>::op(-ai[i], bi[j], accr[i][j]);
                        acci[i][j] = Mfma<T>::op(ai[i], br[j], acci[i][j]);
                    }
            }
        }
        if (more) lstore(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
    // epilogue: element e of a lane is row Mfma<T>::row(lane, e), column lane % 16
    // of its 16x16 block (operands: A[lane % 16][lane / 16], B[lane / 16][lane % 16])
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = m0 + wm * 16 * WM + i * 16 + Mfma<T>::row(lane, e);
                const int col = n0 + wn * 16 * WN + j * 16 + (lane & 15);
                if (row < M && col < N) {
                    GT *pc = C + ((int64_t)row * ldc + col) * ec;
                    T vr, vi;
                    if constexpr (M3) {
                        vr = alpha * (accr[i][j][e] - acci[i][j][e]);
                        vi = alpha * (accs[i][j][e] - accr[i][j][e] - acci[i][j][e]);
                    } else {
                        vr = alpha * accr[i][j][e];
                        vi = alpha * acci[i][j][e];
                    }
                    if (beta != T(0)) {
                        vr += beta * pc[0];
                        if constexpr (CC) vi += beta * pc[1];
                    }
                    if (add_eye && row == col) vr += T(1);
                    pc[0] = vr;
                    if constexpr (CC) pc[1] = vi;
                    if constexpr (MIR) {
                        if (row >= 1) {
                            GT *pm = C + (col - (int64_t)row * ldc) * ec;
                            pm[0] = vr;
                            pm[1] = -vi;
                        }
                    }
                    if (C32) {
                        float *q = C32 + ((int64_t)row * ldc + col) * 2;
                        q[0] = (float)vr;
                        q[1] = (float)vi;
                    }
                }
            }
}

// XR: tile order.  0: as launched; 1 and 2: workgroups are dealt to the
// eight XCDs in turn, each with its own L2, so each XCD gets a contiguous
// range of tiles, row band by row band (1: tiles sharing an A row band share
// that XCD's L2) or column band by column band (2: tiles sharing a B column
// band do, for products whose B is much larger than A).
template <typename T, bool AC, bool BC, int WM, int WN, int BK, int OCC, int XR, bool M3 = false, bool MIR = false>
__global__ __launch_bounds__(256, OCC) void k_gemm(int M, int N, int K, T alpha, const T *__restrict__ A, int64_t lda,
                                                 int64_t sA, const T *B, int64_t ldb, int64_t sB, T beta,
                                                 T *C, int64_t ldc, int64_t sC, int add_eye, float *C32,
                                                 int64_t sC32) {
    constexpr int ea = AC ? 2 : 1, eb = BC ? 2 : 1, ec = (AC || BC) ? 2 : 1;
    int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
    if constexpr (XR != 0) {
        const int gx = gridDim.x, gy = gridDim.y;
        const int64_t nt = (int64_t)gx * gy * gridDim.z, l = bx + (int64_t)gx * (by + (int64_t)gy * bz);
        const int64_t n8 = nt / 8, t = l < 8 * n8 ? (l % 8) * n8 + l / 8 : l;
        if constexpr (XR == 1) {
            bx = (int)(t % gx);
            by = (int)((t / gx) % gy);
        } else {
            by = (int)(t % gy);
            bx = (int)((t / gy) % gx);
        }
        bz = (int)(t / ((int64_t)gx * gy));
    }
    A += (int64_t)bz * sA * ea;
    B += (int64_t)bz * sB * eb;
    C += (int64_t)bz * sC * ec;
    if (C32) C32 += (int64_t)bz * sC32 * 2;
    gemm_tile<T, AC, BC, WM, WN, BK, M3, T, MIR>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, add_eye, C32,
                                                 by * 32 * WM, bx * 32 * WN);
}

// Tile t of a multi-product launch: its item (searched from item a up; the
// items are ordered by their first tile) and the tile within it.
template <typename T, bool AC, bool BC, int WM, int WN, int BK, bool M3>
__device__ __forceinline__ void item_tile(const GemmItem *__restrict__ items, int n_items, int64_t t, int &a) {
    constexpr int ea = AC ? 2 : 1, eb = BC ? 2 : 1, ec = (AC || BC) ? 2 : 1;
    int b = n_items - 1;
    while (a < b) {
        const int m = (a + b + 1) >> 1;
        if (items[m].t0 <= t) a = m;
        else b = m - 1;
    }
    const GemmItem g = items[a];
    const int64_t r = t - g.t0, per = (int64_t)g.tx * g.ty;
    const int bz = (int)(r / per);
    const int64_t rr = r - bz * per;
    const int by = (int)(rr / g.tx), bx = (int)(rr % g.tx);
    // operands through global-address-space pointers (see dglobal)
    typedef dglobal<T> GT;
    const GT *Ap = (const GT *)g.A + (int64_t)bz * g.sA * ea;
    const GT *Bp = (const GT *)g.B + (int64_t)bz * g.sB * eb;
    GT *Cp = (GT *)g.C + (int64_t)bz * g.sC * ec;
    gemm_tile<T, AC, BC, WM, WN, BK, M3, GT>(g.M, g.N, g.K, (T)g.alpha, Ap, g.lda, Bp, g.ldb, (T)g.beta, Cp, g.ldc, 0,
                                             nullptr, by * 32 * WM, bx * 32 * WN);
}

// Many products in one launch, one tile per workgroup, the hardware
// dispatcher handing out the tiles: workgroup l (dealt to XCD l mod 8) takes
// tile (l mod 8) n/8 + l/8, so each XCD works through a contiguous run of
// tiles (consecutive tiles share an A row band, in that XCD's L2).
template <typename T, bool AC, bool BC, int WM, int WN, int BK, int OCC, bool M3>
__global__ __launch_bounds__(256, OCC) void k_gemm_group(const GemmItem *__restrict__ items, int n_items,
                                                       int64_t n_tiles) {
    const int64_t l = blockIdx.x, n8 = n_tiles / 8;
    const int64_t t = l < 8 * n8 ? (l % 8) * n8 + l / 8 : l;
    int a = 0;
    item_tile<T, AC, BC, WM, WN, BK, M3>(items, n_items, t, a);
}

// Workgroup barrier that orders LDS accesses only: unlike __syncthreads it
// does not wait for outstanding global stores (a tile's results) to land.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
}

// Persistent form of the same: the tiles are handed out by eight work queues,
// queue q owning the tiles [q n / 8, (q + 1) n / 8) in order.  A workgroup
// pulls from the queue of its XCD (workgroups are dealt to the XCDs in turn),
// then from the others; it leaves when all eight are empty, so every
// workgroup ends.  queue: eight counters, zero at launch.  On the LU's
// products it runs about a tenth slower than k_gemm_group, most likely
// because a wave's memory operations complete in order: the first loads of a
// workgroup's next tile wait for its previous tile's result stores to drain,
// which a newly dispatched workgroup does not.
template <typename T, bool AC, bool BC, int WM, int WN, int BK, int OCC, bool M3>
__global__ __launch_bounds__(256, OCC) void k_gemm_queue(const GemmItem *__restrict__ items, int n_items,
                                                       int64_t n_tiles, unsigned *__restrict__ queue) {
    __shared__ int64_t s_t;
    const int home = blockIdx.x & 7;
    for (int k = 0; k < 8; ++k) {
        const int q = (home + k) & 7;
        const int64_t lo = n_tiles * q / 8, hi = n_tiles * (q + 1) / 8;
        __syncthreads();  // everyone has read s_t
        if (threadIdx.x == 0) s_t = lo + (int64_t)atomicAdd(&queue[q], 1u);
        __syncthreads();
        int a = 0;  // item of the previous tile: one workgroup's tiles of a queue only grow
        for (;;) {
            // uniform over the workgroup: keep the tile index, the item
            // search and the item's fields in scalar registers
            const int64_t tv = s_t;
            const int64_t t = ((int64_t)__builtin_amdgcn_readfirstlane((int)(tv >> 32)) << 32) |
                              (unsigned)__builtin_amdgcn_readfirstlane((int)tv);
            if (t >= hi) break;
            // the next pull goes out now; its latency hides behind this
            // tile's first loads
            unsigned nxt = 0;
            if (threadIdx.x == 0) nxt = atomicAdd(&queue[q], 1u);
            item_tile<T, AC, BC, WM, WN, BK, M3>(items, n_items, t, a);
            lds_barrier();  // everyone has read s_t; the tile is done with LDS
            if (threadIdx.x == 0) s_t = lo + (int64_t)nxt;
            lds_barrier();
        }
    }
}

// ------------------------------------------------------------------ split-BF16 complex GEMM
// C = alpha A B + beta C for complex float, on v_mfma_f32_16x16x32_bf16: every
// float x is split into three bf16 terms x = h + m + l (round to nearest even
// at each step, so each remainder is exact in float), and the six products
// with h h, h m, m h, h l, m m, l h are accumulated in float.  The neglected
// terms are below 2^-24 relative, so the result is as accurate as an FP32
// product while running on the BF16 matrix rate.  Operand layout (measured on
// gfx950): lane l holds A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16],
// i = 0..7; result element r of lane l is D[4 (l / 16) + r][l % 16].
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline unsigned short bf16_rne(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf16_to_f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

constexpr int XK = 32;  // complex k per stage

__global__ __launch_bounds__(256, 1) void k_cgemm_bf16x(int M, int N, int K, float alpha, const float *__restrict__ A,
                                                        int64_t lda, int64_t sA, const float *B, int64_t ldb,
                                                        int64_t sB, float beta, float *C, int64_t ldc, int64_t sC) {
    // planes [term 0..2][part re/im][row or col 0..63][k 0..31] of bf16
    __shared__ unsigned short As[3][2][64][XK];
    __shared__ unsigned short Bs[3][2][64][XK];
    const int bz = blockIdx.z;
    A += (int64_t)bz * sA * 2;
    B += (int64_t)bz * sB * 2;
    C += (int64_t)bz * sC * 2;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    f32x4 arr[2][2], aii[2][2], ari[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) arr[i][j] = aii[i][j] = ari[i][j] = f32x4{0, 0, 0, 0};
    // staging: A thread (row = tid / 4, k = (tid % 4) * 8 .. +8); B thread (col = tid % 64, k = (tid / 64) * 8 .. +8)
    const int a_row = tid >> 2, a_k = (tid & 3) * 8;
    const int b_col = tid & 63, b_k = (tid >> 6) * 8;
    float ar[8], ai[8], br[8], bi[8];
    auto gload = [&](int k0) {
        const int gr = m0 + a_row;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int gk = k0 + a_k + c;
            if (gr < M && gk < K) {
                const float *p = A + ((int64_t)gr * lda + gk) * 2;
                ar[c] = p[0];
                ai[c] = p[1];
            } else {
                ar[c] = 0.f;
                ai[c] = 0.f;
            }
        }
        const int gc = n0 + b_col;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int gk = k0 + b_k + c;
            if (gc < N && gk < K) {
                const float *p = B + ((int64_t)gk * ldb + gc) * 2;
                br[c] = p[0];
                bi[c] = p[1];
            } else {
                br[c] = 0.f;
                bi[c] = 0.f;
            }
        }
    };
    auto split_store = [&](unsigned short (*P)[2][64][XK], int part, int rc, int k, const float *x) {
        unsigned short h[8], mm[8], l[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            h[c] = bf16_rne(x[c]);
            const float r1 = x[c] - bf16_to_f(h[c]);
            mm[c] = bf16_rne(r1);
            l[c] = bf16_rne(r1 - bf16_to_f(mm[c]));
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            P[0][part][rc][k + c] = h[c];
            P[1][part][rc][k + c] = mm[c];
            P[2][part][rc][k + c] = l[c];
        }
    };
    gload(0);
    for (int k0 = 0; k0 < K; k0 += XK) {
        __syncthreads();
        split_store(As, 0, a_row, a_k, ar);
        split_store(As, 1, a_row, a_k, ai);
        split_store(Bs, 0, b_col, b_k, br);
        split_store(Bs, 1, b_col, b_k, bi);
        __syncthreads();
        if (k0 + XK < K) gload(k0 + XK);
        // B fragments of all three terms for both column blocks
        bf16x8 fb[3][2][2];  // [term][part][block j]
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
            for (int part = 0; part < 2; ++part)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    fb[t][part][j] = *reinterpret_cast<const bf16x8 *>(
                        &Bs[t][part][wn * 32 + j * 16 + (lane & 15)][8 * (lane >> 4)]);
        // A term t pairs with B terms q, t + q <= 2
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            bf16x8 fa[2][2];  // [part][block i]
#pragma unroll
            for (int part = 0; part < 2; ++part)
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    fa[part][i] = *reinterpret_cast<const bf16x8 *>(
                        &As[t][part][wm * 32 + i * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (t + q > 2) continue;
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        arr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[q][0][j], arr[i][j], 0, 0, 0);
                        aii[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[1][i], fb[q][1][j], aii[i][j], 0, 0, 0);
                        ari[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][i], fb[q][1][j], ari[i][j], 0, 0, 0);
                        ari[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[1][i], fb[q][0][j], ari[i][j], 0, 0, 0);
                    }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + e;
                const int col = n0 + wn * 32 + j * 16 + (lane & 15);
                if (row < M && col < N) {
                    float *pc = C + ((int64_t)row * ldc + col) * 2;
                    float vr = alpha * (arr[i][j][e] - aii[i][j][e]);
                    float vi = alpha * ari[i][j][e];
                    if (beta != 0.f) {
                        vr += beta * pc[0];
                        vi += beta * pc[1];
                    }
                    pc[0] = vr;
                    pc[1] = vi;
                }
            }
}

// A = 1 - diag(lam) chi0 (compressed metric), optional complex-float copy.
// Grid: x = 256-column blocks, y = rows, z = batch entries (grid strides).
__global__ void k_formA_diag(int n, int batch, const double *__restrict__ lam, const zdbl *__restrict__ chi0,
                             int64_t s_chi, zdbl *__restrict__ A, int64_t s_A, zflt *A32, int64_t s_A32) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    for (int b = blockIdx.z; b < batch; b += gridDim.z)
        for (int i = blockIdx.y; i < n; i += gridDim.y) {
            const int64_t idx = (int64_t)i * n + j;
            const zdbl c = chi0[b * s_chi + idx];
            zdbl a{-lam[i] * c.re, -lam[i] * c.im};
            if (i == j) a.re += 1.0;
            A[b * s_A + idx] = a;
            if (A32) A32[b * s_A32 + idx] = zflt{(float)a.re, (float)a.im};
        }
}

// Tile of the long complex products (M >= 256, K >= 128): < 0 the default
// (FP64 128x32, FP32 128x64); 0: 64x64 K16; 1: 128x64 K8; 2: 64x32 K8;
// 3: 128x32 K8.  Per host thread, so the batched driver can record each
// molecule with its tuned tile.  Thin complex FP64 products always take 64x32.
thread_local int g_gemm_tile = -1;

const char *const kZgemmName[4] = {"zgemm_64x64", "zgemm_128x64", "zgemm_64x32", "zgemm_128x32"};
const char *const kCgemmName[4] = {"cgemm_64x64", "cgemm_128x64", "cgemm_64x32", "cgemm_128x32"};
const char *const kZgemm3Name[4] = {"zgemm3m_64x64", "zgemm3m_128x64", "zgemm3m_64x32", "zgemm3m_128x32"};

template <typename T, bool AC, bool BC, bool M3 = false>
hipError_t launch_gemm_t(hipStream_t st, int M, int N, int K, T alpha, const T *A, int64_t lda, int64_t sA,
                         const T *B, int64_t ldb, int64_t sB, T beta, T *C, int64_t ldc, int64_t sC, int batch,
                         int add_eye = 0, float *C32 = nullptr, int64_t sC32 = 0) {
    if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
    constexpr bool Z64 = AC && BC && sizeof(T) == 8;
    constexpr bool CF32 = AC && BC && sizeof(T) == 4;
    const bool tuned = g_gemm_tile >= 0 && g_gemm_tile <= 3;
    int tile;
    if constexpr (Z64) {
        const bool big = M >= 256 && K >= 128;
        // the three-product form takes 64x32 at five waves per SIMD by
        // default, for long and thin products alike (68 TF on the LU and solve
        // products at 2000 rows, against 65 TF for the four-product 128x32)
        tile = big ? (tuned ? g_gemm_tile : (M3 ? 2 : 3)) : 2;
        if (M3 && tile == 1) tile = 3;  // 128x64 with a third accumulator would spill
    } else if constexpr (CF32) {
        const bool big = M >= 256 && K >= 128;
        tile = big && tuned ? g_gemm_tile : (M >= 128 && K >= 64) ? 1 : 0;
    } else {
        tile = 0;
    }
    if (OpRecorder *rec = g_rec) {
        // lock-step recording: complex products become work-queue items, the
        // rest run as they are when their lock step comes
        if constexpr (Z64 || CF32) {
            RecOp o;
            o.kind = RecOp::GEMM;
            o.key = (Z64 ? (M3 ? QK_Z3M : QK_Z4M) : QK_C) * 4 + tile;
            o.g.A = A;
            o.g.B = B;
            o.g.C = C;
            o.g.lda = lda;
            o.g.ldb = ldb;
            o.g.ldc = ldc;
            o.g.sA = sA;
            o.g.sB = sB;
            o.g.sC = sC;
            o.g.alpha = (double)alpha;
            o.g.beta = (double)beta;
            o.g.M = M;
            o.g.N = N;
            o.g.K = K;
            o.g.batch = batch;
            o.flops = 8.0 * M * N * (double)K * batch;
            if (!add_eye && !C32) {
                rec->ops.push_back(std::move(o));
                return hipSuccess;
            }
        }
        rec->other([=](hipStream_t s2) {
            return launch_gemm_t<T, AC, BC, M3>(s2, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch,
                                                add_eye, C32, sC32);
        });
        return hipSuccess;
    }
    ProfSink *prof = g_prof;
    const char *cls = nullptr;
    double flops = 0, bytes = 0;
    if (prof) {
        const bool dbl = sizeof(T) == 8;
        if (AC && BC) cls = dbl ? (M3 ? kZgemm3Name[tile] : kZgemmName[tile]) : kCgemmName[tile];
        else if (BC) cls = add_eye ? "formA" : "dzgemm";
        else if (AC) cls = "zdgemm";
        else cls = "dgemm";
        const double ea = sizeof(T) * (AC ? 2 : 1), eb = sizeof(T) * (BC ? 2 : 1), ec = sizeof(T) * ((AC || BC) ? 2 : 1);
        flops = (AC && BC ? 8.0 : (AC || BC) ? 4.0 : 2.0) * M * N * (double)K * batch;
        bytes = (double)M * K * ea * (sA ? batch : 1) + (double)K * N * eb * (sB ? batch : 1) +
                (double)M * N * ec * batch * (beta != T(0) ? 2 : 1);
    }
    ProfScope ps(st, cls ? cls : "", flops, bytes);
#define GW_GEMM(WM, WN, BK, OCC, XR)                                                                               \
    hipLaunchKernelGGL((k_gemm<T, AC, BC, WM, WN, BK, OCC, XR, M3>), dim3((N + 32 * WN - 1) / (32 * WN),           \
                       (M + 32 * WM - 1) / (32 * WM), batch), dim3(256), 0, st, M, N, K, alpha, A, lda, sA, B, ldb, \
                       sB, beta, C, ldc, sC, add_eye, C32, sC32)
    if constexpr (Z64 || CF32) {
        // the three-product 128x32 tile needs a third accumulator: three
        // workgroups per CU instead of four, so that nothing spills
        if (tile == 3) GW_GEMM(4, 1, 8, M3 ? 3 : 4, true);
        else if (tile == 2) GW_GEMM(2, 1, 8, M3 ? 5 : 4, true);
        else if (tile == 1) GW_GEMM(4, 2, 8, 2, false);
        else GW_GEMM(2, 2, 16, 2, false);
    } else {
        if (tile == 1) GW_GEMM(4, 2, 8, 2, false);
        else GW_GEMM(2, 2, 16, 2, false);
    }
#undef GW_GEMM
    return hipGetLastError();
}

}  // namespace

hipError_t launch_zgemm(hipStream_t st, int M, int N, int K, double alpha, const zdbl *A, int64_t lda, int64_t sA,
                        const zdbl *B, int64_t ldb, int64_t sB, double beta, zdbl *C, int64_t ldc, int64_t sC,
                        int batch) {
    return launch_gemm_t<double, true, true>(st, M, N, K, alpha, (const double *)A, lda, sA, (const double *)B, ldb,
                                             sB, beta, (double *)C, ldc, sC, batch);
}

// The products of the FP64 LU and solves: the three-product form.
hipError_t launch_zgemm_lu(hipStream_t st, int M, int N, int K, double alpha, const zdbl *A, int64_t lda,
                           int64_t sA, const zdbl *B, int64_t ldb, int64_t sB, double beta, zdbl *C, int64_t ldc,
                           int64_t sC, int batch) {
    return launch_gemm_t<double, true, true, true>(st, M, N, K, alpha, (const double *)A, lda, sA, (const double *)B,
                                                   ldb, sB, beta, (double *)C, ldc, sC, batch);
}

// C = alpha A B (beta = 0) for complex A (M x K, small) times real B (K x N,
// N large), tiles ordered column band by column band so each slice of B is
// read from HBM once: the Cauchy transform of the spectral bins on the
// A route (M frequencies, N matrix entries, K bins).  mirror: row r >= 1 is
// also written, conjugated, at row -r (C's rows are the mesh points from
// omega = 0 up; the rows before C are those of -omega).
hipError_t launch_zdgemm_wide(hipStream_t st, int M, int N, int K, double alpha, const zdbl *A, int64_t lda,
                              const double *B, int64_t ldb, zdbl *C, int64_t ldc, bool mirror) {
    if (M <= 0 || N <= 0) return hipSuccess;
    ProfScope ps(st, "cauchy_gemm", 4.0 * M * (double)N * K,
                 8.0 * (double)K * N + 16.0 * (double)(mirror ? 2 * M - 1 : M) * N);
    const dim3 grid((N + 63) / 64, (M + 63) / 64, 1);
    if (mirror)
        hipLaunchKernelGGL((k_gemm<double, true, false, 2, 2, 16, 2, 2, false, true>), grid, dim3(256), 0, st, M, N, K,
                           alpha, (const double *)A, lda, (int64_t)0, B, ldb, (int64_t)0, 0.0, (double *)C, ldc,
                           (int64_t)0, 0, (float *)nullptr, (int64_t)0);
    else
        hipLaunchKernelGGL((k_gemm<double, true, false, 2, 2, 16, 2, 2>), grid, dim3(256), 0, st, M, N, K, alpha,
                           (const double *)A, lda, (int64_t)0, B, ldb, (int64_t)0, 0.0, (double *)C, ldc, (int64_t)0,
                           0, (float *)nullptr, (int64_t)0);
    return hipGetLastError();
}

// Complex-float products of the calling thread run as split-BF16 MFMA when set
// (the trailing updates of the BF16x LU).
thread_local bool g_cgemm_bf16x = false;

hipError_t launch_cgemm(hipStream_t st, int M, int N, int K, float alpha, const zflt *A, int64_t lda, int64_t sA,
                        const zflt *B, int64_t ldb, int64_t sB, float beta, zflt *C, int64_t ldc, int64_t sC,
                        int batch) {
    if (g_cgemm_bf16x && K >= 32) {
        if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
        if (OpRecorder *rec = g_rec) {
            rec->other([=](hipStream_t s2) {
                OpRecorder *saved = g_rec;
                g_rec = nullptr;
                const bool prev = g_cgemm_bf16x;
                g_cgemm_bf16x = true;
                const hipError_t e = launch_cgemm(s2, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch);
                g_cgemm_bf16x = prev;
                g_rec = saved;
                return e;
            });
            return hipSuccess;
        }
        dim3 grid((N + 63) / 64, (M + 63) / 64, batch);
        ProfScope ps(st, "cgemm_bf16x", 8.0 * M * N * (double)K * batch,
                     8.0 * ((double)M * K + (double)K * N + (beta != 0.f ? 2.0 : 1.0) * M * N) * batch);
        hipLaunchKernelGGL(k_cgemm_bf16x, grid, dim3(256), 0, st, M, N, K, alpha, (const float *)A, lda, sA,
                           (const float *)B, ldb, sB, beta, (float *)C, ldc, sC);
        return hipGetLastError();
    }
    return launch_gemm_t<float, true, true>(st, M, N, K, alpha, (const float *)A, lda, sA, (const float *)B, ldb, sB,
                                            beta, (float *)C, ldc, sC, batch);
}

hipError_t launch_formA(hipStream_t st, int n, const double *v, int v_is_diag, const zdbl *chi0, int64_t s_chi,
                        zdbl *A, int64_t s_A, zflt *A32, int64_t s_A32, int batch) {
    if (v_is_diag) {
        GW_DEFER(launch_formA(st, n, v, v_is_diag, chi0, s_chi, A, s_A, A32, s_A32, batch));
        const int xb = (n + 255) / 256, zb = std::min(batch, 65535);
        dim3 grid((unsigned)xb, (unsigned)std::max(1, std::min(n, 65536 / std::max(1, xb * zb))), (unsigned)zb);
        hipLaunchKernelGGL(k_formA_diag, grid, dim3(256), 0, st, n, batch, v, chi0, s_chi, A, s_A, A32, s_A32);
        return hipGetLastError();
    }
    // A = -v * chi0 + 1 (v real, shared by the batch: batch stride 0)
    return launch_gemm_t<double, false, true>(st, n, n, n, -1.0, v, n, 0, (const double *)chi0, n, s_chi, 0.0,
                                              (double *)A, n, s_A, batch, 1, (float *)A32, s_A32);
}

// R = v - A W: R <- v (complex), then R -= A W.
hipError_t launch_residual(hipStream_t st, int n, const double *v, int v_is_diag, const zdbl *A, int64_t sA,
                           const zdbl *W, int64_t sW, zdbl *R, int64_t sR, int batch) {
    hipError_t e = launch_init_rhs(st, n, v, v_is_diag, R, sR, batch);
    if (e != hipSuccess) return e;
    return launch_zgemm(st, n, n, n, -1.0, A, n, sA, W, n, sW, 1.0, R, n, sR, batch);
}

// Real-times-complex and complex-times-real products exposed for the compression path.
hipError_t launch_dzgemm(hipStream_t st, int M, int N, int K, double alpha, const double *A, int64_t lda, int64_t sA,
                         const zdbl *B, int64_t ldb, int64_t sB, double beta, zdbl *C, int64_t ldc, int64_t sC,
                         int batch) {
    return launch_gemm_t<double, false, true>(st, M, N, K, alpha, A, lda, sA, (const double *)B, ldb, sB, beta,
                                              (double *)C, ldc, sC, batch);
}
hipError_t launch_zdgemm(hipStream_t st, int M, int N, int K, double alpha, const zdbl *A, int64_t lda, int64_t sA,
                         const double *B, int64_t ldb, int64_t sB, double beta, zdbl *C, int64_t ldc, int64_t sC,
                         int batch) {
    return launch_gemm_t<double, true, false>(st, M, N, K, alpha, (const double *)A, lda, sA, B, ldb, sB, beta,
                                              (double *)C, ldc, sC, batch);
}
hipError_t launch_dgemm(hipStream_t st, int M, int N, int K, double alpha, const double *A, int64_t lda, int64_t sA,
                        const double *B, int64_t ldb, int64_t sB, double beta, double *C, int64_t ldc, int64_t sC,
                        int batch) {
    return launch_gemm_t<double, false, false>(st, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch);
}

thread_local OpRecorder *g_rec = nullptr;

namespace {
// (WM, WN, BK, OCC) of each work-queue key: the tiles and occupancies
// launch_gemm_t picks for the product kind and tile.  The queue loop keeps a
// few per-lane addresses live across tiles; at these occupancies the
// three-product tiles (64x32 at five, 128x32 at three per CU) move them to
// scratch memory, reloaded once per tile, never in the K loop.
struct QShape {
    int wm, wn, bk, occ;
};
QShape qshape(int key) {
    const int kind = key / 4, tile = key % 4;
    if (kind == QK_Z3M) {
        if (tile == 2) return {2, 1, 8, 5};
        if (tile == 0) return {2, 2, 16, 2};
        return {4, 1, 8, 3};  // 3 (and 1, which maps to it)
    }
    if (tile == 3) return {4, 1, 8, kind == QK_C ? 4 : 3};  // four-product 128x32 at four would use AGPRs
    if (tile == 2) return {2, 1, 8, 4};
    if (tile == 1) return {4, 2, 8, 2};
    return {2, 2, 16, 2};
}
}  // namespace

int gemm_queue_occupancy(int key) {
    // workgroups of this key resident on one CU, as the runtime computes it
    // from the kernel's registers and LDS (at least the launch bound's figure)
    int occ = 0;
    hipError_t e = hipErrorInvalidValue;
    const int kind = key / 4, tile = key % 4;
#define GW_QOCC(T, M3, WM, WN, BK, OCC) \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_gemm_queue<T, true, true, WM, WN, BK, OCC, M3>, 256, 0)
    if (kind == QK_Z3M) {
        if (tile == 2) GW_QOCC(double, true, 2, 1, 8, 5);
        else if (tile == 0) GW_QOCC(double, true, 2, 2, 16, 2);
        else GW_QOCC(double, true, 4, 1, 8, 3);
    } else if (kind == QK_Z4M) {
        if (tile == 3) GW_QOCC(double, false, 4, 1, 8, 3);
        else if (tile == 2) GW_QOCC(double, false, 2, 1, 8, 4);
        else if (tile == 1) GW_QOCC(double, false, 4, 2, 8, 2);
        else GW_QOCC(double, false, 2, 2, 16, 2);
    } else {
        if (tile == 3) GW_QOCC(float, false, 4, 1, 8, 4);
        else if (tile == 2) GW_QOCC(float, false, 2, 1, 8, 4);
        else if (tile == 1) GW_QOCC(float, false, 4, 2, 8, 2);
        else GW_QOCC(float, false, 2, 2, 16, 2);
    }
#undef GW_QOCC
    return e == hipSuccess && occ > 0 ? occ : qshape(key).occ;
}
void gemm_queue_tile(int key, int *bm, int *bn) {
    const QShape q = qshape(key);
    *bm = 32 * q.wm;
    *bn = 32 * q.wn;
}

hipError_t launch_gemm_queue(hipStream_t st, int key, const GemmItem *items, int n_items, int64_t n_tiles,
                             unsigned *queue, int grid, double flops) {
    if (n_items <= 0 || n_tiles <= 0) return hipSuccess;
    if (key < 0 || key >= 12 || (!queue && n_tiles > INT32_MAX) || (queue && grid <= 0)) return hipErrorInvalidValue;
    const int kind = key / 4, tile = key % 4;
    static const char *const names[3] = {"zgemm3m_queue", "zgemm_queue", "cgemm_queue"};
    ProfScope ps(st, names[kind], flops, 0.0);
#define GW_QGEMM(T, M3, WM, WN, BK, OCC)                                                                        \
    do {                                                                                                         \
        if (queue)                                                                                               \
            hipLaunchKernelGGL((k_gemm_queue<T, true, true, WM, WN, BK, OCC, M3>), dim3(grid), dim3(256), 0, st, \
                               items, n_items, n_tiles, queue);                                                  \
        else                                                                                                     \
            hipLaunchKernelGGL((k_gemm_group<T, true, true, WM, WN, BK, OCC, M3>), dim3((unsigned)n_tiles),      \
                               dim3(256), 0, st, items, n_items, n_tiles);                                       \
    } while (0)
    if (kind == QK_Z3M) {
        if (tile == 2) GW_QGEMM(double, true, 2, 1, 8, 5);
        else if (tile == 0) GW_QGEMM(double, true, 2, 2, 16, 2);
        else GW_QGEMM(double, true, 4, 1, 8, 3);
    } else if (kind == QK_Z4M) {
        if (tile == 3) GW_QGEMM(double, false, 4, 1, 8, 3);
        else if (tile == 2) GW_QGEMM(double, false, 2, 1, 8, 4);
        else if (tile == 1) GW_QGEMM(double, false, 4, 2, 8, 2);
        else GW_QGEMM(double, false, 2, 2, 16, 2);
    } else {
        if (tile == 3) GW_QGEMM(float, false, 4, 1, 8, 4);
        else if (tile == 2) GW_QGEMM(float, false, 2, 1, 8, 4);
        else if (tile == 1) GW_QGEMM(float, false, 4, 2, 8, 2);
        else GW_QGEMM(float, false, 2, 2, 16, 2);
    }
#undef GW_QGEMM
    return hipGetLastError();
}

}  // namespace gwk

namespace gwp {
void set_thread_gemm_tile(int tile) { gwk::g_gemm_tile = tile; }
bool set_thread_cgemm_bf16x(bool on) {
    const bool prev = gwk::g_cgemm_bf16x;
    gwk::g_cgemm_bf16x = on;
    return prev;
}
}  // namespace gwp
