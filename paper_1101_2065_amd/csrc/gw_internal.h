// Internal declarations shared by the HIP translation units of libgw.so.
// Host-side launchers for every kernel, plus small device helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <vector>

namespace gwk {

struct zdbl {
    double re, im;
};
struct zflt {
    float re, im;
};

// ---------------------------------------------------------------- lock-step recording
// One batched product C = alpha A B + beta C of a work-queue launch (device
// readable): tx x ty tiles per batch entry, tiles t0 .. t0 + tx ty batch - 1
// of the launch.
struct GemmItem {
    const void *A, *B;
    void *C;
    int64_t lda, ldb, ldc, sA, sB, sC;
    double alpha, beta;
    int M, N, K, batch;
    int tx, ty;
    int64_t t0;
};
// One batched panel factorisation or row-exchange pass of a grouped launch:
// its workgroups are wg0 .. wg0 + count - 1 of the launch.
struct PanelItem {
    void *A;
    int64_t sA;
    int32_t *ipiv, *swp, *info;
    void *Linv, *Uinv;
    int n, kb, w, nblk, batch;
    int64_t wg0;
};
// While a recorder is installed on the calling host thread, the launchers of
// the W solve append their work to it instead of launching (the batched
// driver runs the recorded programs of many molecules in lock step).
// kind: GEMM (key = product kind * 4 + tile), PANEL (key = panel variant),
// LASWP (key = 0 double, 1 float), OTHER (run fn on the lock step's stream),
// MARK (the factorisation or a substitution starts or ends).
struct RecOp {
    enum Kind { GEMM, PANEL, LASWP, OTHER, MARK } kind;
    int key = 0;
    GemmItem g{};
    PanelItem p{};
    double flops = 0;
    std::function<hipError_t(hipStream_t)> fn;
};
struct OpRecorder {
    std::vector<RecOp> ops;
    void other(std::function<hipError_t(hipStream_t)> f) {
        RecOp o;
        o.kind = RecOp::OTHER;
        o.fn = std::move(f);
        ops.push_back(std::move(o));
    }
    void mark() {
        RecOp o;
        o.kind = RecOp::MARK;
        ops.push_back(std::move(o));
    }
};
extern thread_local OpRecorder *g_rec;
// Element type for device pointers read from a descriptor in memory: the
// global address space in the device compilation (the compiler cannot infer it
// for a loaded pointer as it does for a kernel argument, and would emit flat
// accesses, whose waits also stall on LDS traffic); the host pass only checks
// the kernels and takes the plain type.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename P>
using dglobal = __attribute__((address_space(1))) P;
#else
template <typename P>
using dglobal = P;
#endif
// In a launcher: while a recorder is installed, run `call` (with `st` its
// stream) when the recorded program reaches it, instead of now.
#define GW_DEFER(call)                                                  \
    do {                                                                \
        if (::gwk::OpRecorder *rec_ = ::gwk::g_rec) {                   \
            rec_->other([=](hipStream_t st) { return call; });          \
            return hipSuccess;                                          \
        }                                                               \
    } while (0)
// product kinds of the work-queue launch
enum { QK_Z3M = 0, QK_Z4M = 1, QK_C = 2 };
// One launch of `n_items` products (descriptors on the device), `n_tiles`
// tiles in all: with `queue` (eight counters, zero) a persistent grid of
// `grid` workgroups pulling tiles from per-XCD work queues, without it one
// workgroup per tile handed out by the hardware dispatcher.
hipError_t launch_gemm_queue(hipStream_t st, int key, const GemmItem *items, int n_items, int64_t n_tiles,
                             unsigned *queue, int grid, double flops);
// Device-to-device copy on `st` (deferred like the kernels while recording).
hipError_t launch_copy(hipStream_t st, void *dst, const void *src, size_t bytes);
// Grouped panel and row-exchange launches over many batched passes.
hipError_t launch_panel_group(hipStream_t st, int key, const PanelItem *items, int n_items, int64_t n_wg);
hipError_t launch_laswp_group(hipStream_t st, int key, const PanelItem *items, int n_items, int64_t n_wg);
// Resident workgroups per CU of a work-queue launch of this key, and the
// tile shape (rows, columns) of its tiles.
int gemm_queue_occupancy(int key);
void gemm_queue_tile(int key, int *bm, int *bn);

// ---------------------------------------------------------------- chi0 build
// Pair vertex (Section 7.A): P[mu][(E-e0)*n_virt + F'] = sum_a X_a^E sum_b V_mu^{ab} X_b^{n_occ+F'}
// for occupied E in [e0, e0+ecnt); rows of P are ldp apart.
hipError_t launch_pairvec(hipStream_t st, int n_orb, int n_occ, int n_prod, int n_blk,
                          const double *X, const int32_t *blk_prod, const int32_t *blk_orb,
                          const int32_t *orb_idx, const int64_t *blk_val, const double *vals,
                          int max_o, int e0, int ecnt, int64_t ldp, double *P);

// Pair bins on the mesh and the bin-sorted pair order (Sections 5, 5.A).
// lo: [n_occ][nhb+1] int32, rowoff: [n_occ][nhb] int32, binoff: [nhb] int32,
// perm: [n_pairs] int32, fsort: [n_pairs] double, stat: [4] int64 (n_kept, n_dropped).
hipError_t launch_pair_sort(hipStream_t st, int n_orb, int n_occ, const double *eig, int kbits,
                            int nhb, int32_t *lo, int32_t *rowoff, int32_t *binoff,
                            int32_t *perm, double *fsort, int64_t *stat);

// Ps[r][i] = P[r][perm[i]], i < n_kept (n_kept read from stat[0]).
hipError_t launch_gather(hipStream_t st, int rows, int64_t n_pairs, const double *P,
                         const int32_t *perm, const int64_t *stat, double *Ps);

// vmax bits (as uint64) of max |P| into dst (must be zeroed first, done inside).
hipError_t launch_absmax(hipStream_t st, const double *P, int64_t n, uint64_t *dst);

// s from the overflow rule (and the caller's request): params[0] = s.
hipError_t launch_fracbits(hipStream_t st, const uint64_t *vmax_bits, int64_t n_pairs,
                           int requested, int32_t *s_out);

hipError_t launch_fill_u64(hipStream_t st, uint64_t *p, int64_t n, uint64_t value);
// A route: A[j] = 1 - (T X)[j] for all j from the products X = v a0 of the
// bins ([nhb][n][n] real, bin row 0 is overwritten with the identity), by one
// complex-times-real product over the solved half of the mesh that also writes
// the conjugate mirror (T: workspace of (n_omega/2 + 1) nhb complex), and the
// lone point j = 0.
hipError_t launch_cauchy_A(hipStream_t st, int n, int n_omega, int nhb, int j0, double domega, double eps,
                           double *X, zdbl *T, zdbl *A);
hipError_t launch_zdgemm_wide(hipStream_t st, int M, int N, int K, double alpha, const zdbl *A, int64_t lda,
                              const double *B, int64_t ldb, zdbl *C, int64_t ldc, bool mirror);
hipError_t launch_fill_u32(hipStream_t st, uint32_t *p, int64_t n, uint32_t value);

// Exact int64 histogram H[nhb][n_upper] (Section 5.A eq. chi_by_spectra).
// With a bin range, only pairs whose lower bin lies in [bin_lo, bin_hi) are
// counted and only rows [bin_lo, bin_hi] of H are written (cleared first);
// bin_hi < 0 means nhb - 1, i.e. every kept pair.
hipError_t launch_hist(hipStream_t st, int n, int64_t n_pairs_cap, const double *Ps,
                       const double *fsort, const int32_t *binoff, const int64_t *stat,
                       const int32_t *s_dev, int nhb, int64_t *H, int splits, int bin_lo = 0, int bin_hi = -1,
                       bool clear = true);

// Kernel spectrum Kt[q] = DFT of k(r) = 1/((r + j0) domega + i eps) (wrapped) and
// the twiddle table tw[q] = exp(-2 pi i q / L).
hipError_t launch_kspec(hipStream_t st, int n_omega, int j0, double domega, double eps,
                        zdbl *Kt, zdbl *tw);

// chi0[j][mu][nu] from H by FFT convolution (Section 5.A, 8.A).
// symmetrize = false: the wave-kernel sizes (256 <= 2 n_omega <= 2048) leave
// the strict lower triangle unwritten (launch_symmetrize fills it later).
hipError_t launch_fftconv(hipStream_t st, int n, int n_omega, int nhb, const int64_t *H,
                          const int32_t *s_dev, const zdbl *Kt, const zdbl *tw, zdbl *chi0,
                          bool symmetrize = true);
// The same from a spectral array A[nhb][n_upper] already in floating point.
hipError_t launch_fftconv(hipStream_t st, int n, int n_omega, int nhb, const double *A,
                          const zdbl *Kt, const zdbl *tw, zdbl *chi0, bool symmetrize = true);
// chi0[j][nu][mu] = chi0[j][mu][nu] for mu < nu, all j < n_omega.
hipError_t launch_symmetrize(hipStream_t st, int n, int n_omega, zdbl *chi0);
// D[m - m0][mu][nu] = 2^-s H[m][t(mu, nu)] for bins m0 <= m < m0 + cnt, both
// triangles.
hipError_t launch_expand_bins(hipStream_t st, int n, int m0, int cnt, const int64_t *H, int64_t n_upper,
                              const int32_t *s_dev, double *D);
// The same from a spectral array already in floating point.
hipError_t launch_expand_bins(hipStream_t st, int n, int m0, int cnt, const double *a, int64_t n_upper, double *D);
// A[j] = 1 - sum_m B[m] K_m(omega_j) for dense B[nhb][n][n] = v a0 (bins
// m >= 1 read), every (mu, nu); 256 <= 2 n_omega <= 2048.
hipError_t launch_fftconv_A(hipStream_t st, int n, int n_omega, int nhb, const double *B, const zdbl *Kt,
                            const zdbl *tw, zdbl *A);

// ---------------------------------------------------------------- dense algebra
// Batched complex GEMM, C = alpha*A*B + beta*C, row-major, element strides,
// batch strides in elements.  If C aliases B the caller guarantees M <= 64.
hipError_t launch_zgemm(hipStream_t st, int M, int N, int K, double alpha,
                        const zdbl *A, int64_t lda, int64_t sA,
                        const zdbl *B, int64_t ldb, int64_t sB, double beta,
                        zdbl *C, int64_t ldc, int64_t sC, int batch);
// The same with three real products per complex product (the FP64 LU and
// solves; see k_gemm.hip).
hipError_t launch_zgemm_lu(hipStream_t st, int M, int N, int K, double alpha,
                           const zdbl *A, int64_t lda, int64_t sA,
                           const zdbl *B, int64_t ldb, int64_t sB, double beta,
                           zdbl *C, int64_t ldc, int64_t sC, int batch);
hipError_t launch_cgemm(hipStream_t st, int M, int N, int K, float alpha,
                        const zflt *A, int64_t lda, int64_t sA,
                        const zflt *B, int64_t ldb, int64_t sB, float beta,
                        zflt *C, int64_t ldc, int64_t sC, int batch);

// A = I - v * chi0 (v real [n][n], chi0 complex), batched over frequencies.
// v_is_diag: v holds the diagonal only.
hipError_t launch_formA(hipStream_t st, int n, const double *v, int v_is_diag,
                        const zdbl *chi0, int64_t s_chi, zdbl *A, int64_t s_A,
                        zflt *A32, int64_t s_A32, int batch);

// Right-looking blocked LU with partial pivoting, batched; factors in place,
// ipiv[batch][n] (0-based global rows), Linv/Uinv [batch][n/64 blocks][64][64].
template <typename Z>
hipError_t getrf_batched(hipStream_t st, int n, Z *A, int64_t sA, int32_t *ipiv,
                         Z *Linv, Z *Uinv, Z *scratch, int32_t *info, int batch);
// Solve A X = B with the factors above, B [batch][n][nrhs] in place.
// sym_lower (nrhs == n, X known to be symmetric): the back substitution only
// produces the lower triangle, which is then mirrored into the upper one.
template <typename Z>
hipError_t getrs_batched(hipStream_t st, int n, int nrhs, const Z *LU, int64_t sA,
                         const int32_t *ipiv, const Z *Linv, const Z *Uinv,
                         Z *B, int64_t sB, int batch, bool sym_lower = false);

// B[b] = v (as complex), v dense or diagonal.
hipError_t launch_init_rhs(hipStream_t st, int n, const double *v, int v_is_diag,
                           zdbl *B, int64_t sB, int batch);
// W[n_omega - j] = conj(W[j]) for j in (n_omega/2, n_omega).
hipError_t launch_conj_mirror(hipStream_t st, int64_t nn, int n_omega, zdbl *W);

// Mixed precision helpers.
hipError_t launch_z2c(hipStream_t st, const zdbl *src, zflt *dst, int64_t n);
hipError_t launch_c2z_add(hipStream_t st, const zflt *d, zdbl *W, int64_t n_per, int batch,
                          const int32_t *active);
// Per-batch sum of squares into out[2*b] (|dW|^2) and out[2*b+1] (|W|^2).
hipError_t launch_norms(hipStream_t st, const zflt *dW, const zdbl *W, int64_t n_per, int batch,
                        double *out);
// R = v - A W (FP64), R complex, A complex, W complex; batched.
hipError_t launch_residual(hipStream_t st, int n, const double *v, int v_is_diag,
                           const zdbl *A, int64_t sA, const zdbl *W, int64_t sW,
                           zdbl *R, int64_t sR, int batch);

// Orthonormal basis Q [n][k] of the dominant k-dimensional eigenspace of v and
// S = Q^T v Q [k][k] (shifted subspace iteration); work: compress_work_doubles.
size_t compress_work_doubles(int n, int k);
// Section 7.A subspace: Z [n][k] orthonormal in the Coulomb metric spanning
// the dominant k-dimensional part of the generators X [n][nr], U = v Z and
// (R non-null) R = v - U U^T; work: pair_basis_work_doubles.
size_t pair_basis_work_doubles(int n, int nr, int k);
hipError_t pair_basis(hipStream_t st, int n, int nr, int k, const double *v, const double *X, double *Z, double *U,
                      double *R, double *work, int iters);
// b = a - b over n int64 entries.
hipError_t launch_sub_i64(hipStream_t st, const int64_t *a, int64_t *b, int64_t n);
// chi[j][mu][nu] += sum_{m in [m_lo, nhb)} 2^-s H[m][mu<=nu] K[j][m - m_lo] for
// j < n_om on the upper triangle only (K: [n_om][nhb - m_lo] complex).  Row
// m_lo comes from H_lo ([n_upper]) instead of H when H_lo is non-null.
hipError_t launch_cauchy_add(hipStream_t st, int n, int n_om, int nhb, int m_lo, const int64_t *H,
                             const int64_t *H_lo, const int32_t *s_dev, const zdbl *K, zdbl *chi);
// K[j][m - m_lo] = 1/(w_j - m d + i eps) - 1/(w_j + m d + i eps), w_j = w0 + j dw.
hipError_t launch_cauchy_table(hipStream_t st, int n_om, double w0, double dw, int nhb, int m_lo, double d,
                               double eps, zdbl *K);
// X[mu][j0 + j] = P[mu][src[j0 + j] - base] for j < ncols.
hipError_t launch_gather_cols(hipStream_t st, int rows, int ncols, int64_t ldp, const double *P, const int32_t *src,
                              int64_t base, int j0, double *X, int64_t ldx);
hipError_t compress_basis(hipStream_t st, int n, int k, const double *v, double *Q_out, double *S_out,
                          double *work, int iters);

// C[b] = alpha A[b] B[b] + beta C[b], real FP64, row-major (MFMA).
hipError_t launch_dgemm(hipStream_t st, int M, int N, int K, double alpha, const double *A, int64_t lda, int64_t sA,
                        const double *B, int64_t ldb, int64_t sB, double beta, double *C, int64_t ldc, int64_t sC,
                        int batch);

// ---------------------------------------------------------------- time-domain a0 route
// Largest orbital set of a vertex block on this route (LDS staging).
#define TIME_MAX_ORB 32
// rho[k][a][b] for k < K from levels listed bin by bin (two-bin split).
hipError_t launch_rho_bins(hipStream_t st, int n_orb, int K, const double *X, const int32_t *lev, const double *ph,
                           const int32_t *start, double *rho);
// F [2Q][K] forward cosine/sine rows (F may be null) and G [M][2Q] inverse
// rows for a real sequence (G may be null), length L, Q = L/2 + 1.
hipError_t launch_dft_matrices(hipStream_t st, int L, int Q, int K, double *F, int M, double *G);
// Ahat[2 qq (+1)][t] for time points q0 .. q0 + nq - 1 over the listed block
// pairs (pb1[i] <= pb2[i]); Rp, Rm: [2Q][n_orb^2] transformed densities.
// The pairs are grouped by tile class c = 2 (|O1| > 16) + (|O2| > 16):
// class c holds the pairs class_off[c] .. class_off[c+1] - 1 (host array).
hipError_t launch_time_contract(hipStream_t st, int n_orb, int n_prod, const int *class_off, int q0, int nq,
                                const int32_t *blk_prod, const int32_t *blk_orb, const int32_t *orb_idx,
                                const int64_t *blk_val, const double *vals, const int32_t *pb1, const int32_t *pb2,
                                const double *Rp, const double *Rm, double *Ahat, double flops);

// ---------------------------------------------------------------- self-energy from W
// gam[k][t] = -(domega/pi) Im W[j0 + k][mu][nu], packed upper t, k < n_sb; gam[0] = 0.
hipError_t launch_w_spectral(hipStream_t st, int n, int n_sb, int j0, double domega, const zdbl *W, double *gam);
// dst[t] = src[mu][nu], packed upper t.
hipError_t launch_pack_upper(hipStream_t st, int n, const double *src, double *dst);
// Kp[j][m] = 1/(w_j - m d + i eps), Km[j][m] = 1/(w_j + m d + i eps), w_j = w0 + j d.
hipError_t launch_cauchy_pm(hipStream_t st, int n_om, int M, double w0, double d, double eps, zdbl *Kp, zdbl *Km);
hipError_t launch_scale_copy(hipStream_t st, int64_t n, double alpha, const double *src, double *dst);
// Dyson's equation: Xe = X diag(eig); Hs = H + Sx - Vxc (null terms skipped);
// A[b] = (w_{j0+b} + i eps) 1 - Hs - Sc[j0+b] (Sc may be null), w_j = w0 + j d;
// dos[j0+b] = -(1/pi) Im tr G[b].
hipError_t launch_scale_cols(hipStream_t st, int n, const double *X, const double *eig, double *Xe);
hipError_t launch_static_part(hipStream_t st, int64_t nn, const double *H, const double *Sx, const double *Vxc,
                              double *Hs);
hipError_t launch_dyson_form(hipStream_t st, int n, int j0, int nb, double w0, double d, double eps, const double *Hs,
                             const zdbl *Sc, zdbl *A);
hipError_t launch_trace_dos(hipStream_t st, int n, int j0, int nb, const zdbl *G, int64_t sG, double *dos);
// S+-[2 qq (+1)][a][b] += sum over the listed block pairs of
// sum_{mu nu} gammahat^{mu nu} (V_mu rho+-(t) V_nu)^{ab} (and the transpose for
// B1 < B2), time points q0 .. q0 + nq - 1.  Rm == nullptr: one density only.
// S+- must be cleared by the caller.  Block pairs grouped by tile class as
// for launch_time_contract.
hipError_t launch_sigma_contract(hipStream_t st, int n_orb, int n_prod, const int *class_off, int q0, int nq,
                                 const int32_t *blk_prod, const int32_t *blk_orb, const int32_t *orb_idx,
                                 const int64_t *blk_val, const double *vals, const int32_t *pb1, const int32_t *pb2,
                                 const double *Rp, const double *Rm, const double *Gh, double *Sp, double *Sm,
                                 int max_vblock, double flops);

}  // namespace gwk
