/*
 * gw.h -- C ABI of the MI355X screened-interaction library (libgw.so).
 *
 * The library builds the screened Coulomb interaction of Hedin's GW
 * approximation in a local product basis, following D. Foerster, P. Koval,
 * D. Sanchez-Portal, "An O(N^3) implementation of Hedin's GW approximation for
 * molecules" (arXiv:1101.2065):
 *
 *   1. pair vectors V_mu^{EF} = X_a^E V_mu^{ab} X_b^F       (Section 7.A)
 *   2. spectral function of the free response a0_{mu nu}(s),
 *      histogrammed on the frequency mesh                    (Section 5.A,
 *                                                              eq. chi_by_spectra)
 *   3. chi0(w + i eps) = Cauchy transform of a0, by FFT      (Section 5.A, 8.A)
 *   4. W(w) = (1 - v chi0(w))^{-1} v by dense complex LU      (Section 2 eq.
 *      Coulombscreening, Section 3 eq. tensorform-scr-inter)
 *   5. optional compression to the top-k eigenvectors of v    (Section 7.B)
 *
 * Conventions for every function below:
 *   - Energies in Hartree, measured from the Fermi level: states with index
 *     < n_occ are occupied (E < 0), the rest empty (Section 3).
 *   - Matrices are row-major.  Complex numbers are interleaved {re, im}
 *     doubles (C99 double _Complex layout) or {re, im} floats for complex64.
 *   - Pointers marked DEVICE are HIP device memory of the context's device;
 *     pointers marked HOST are ordinary host memory.  The caller owns every
 *     buffer it passes and must keep it alive until the call returns (for
 *     gw_submit: until gw_poll returns GW_OK for that ticket).
 *   - All GPU work is enqueued on the hipStream_t passed as void* (NULL = the
 *     null stream).  Functions return when the work is enqueued unless they
 *     say otherwise.
 *   - Errors are status codes; nothing throws across the ABI.  Arguments are
 *     checked before anything is launched (GW_E_INVALID).  A device error is
 *     sticky: every later call on that context returns GW_E_DEVICE until
 *     gw_destroy.  gw_last_error() gives a message for the last failure.
 *   - One context per host thread; contexts are not thread-safe, except that
 *     gw_submit / gw_poll / gw_release may be called from any one thread while
 *     the context's serving worker runs.
 */
#ifndef GW_H
#define GW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GW_OK = 0,
    GW_PENDING = 1,     /* gw_poll: not finished yet */
    GW_E_INVALID = -1,  /* bad argument (shape, layout, ordering, grid) */
    GW_E_OOM = -2,      /* device workspace could not be allocated */
    GW_E_DEVICE = -3,   /* HIP runtime or kernel failure (sticky) */
    GW_E_NOCONV = -4,   /* refinement did not converge and fallback disabled */
    GW_E_RANGE = -5,    /* value outside what the fixed-point format can hold */
    GW_E_STATE = -6     /* call not valid in the current state (unknown ticket ...) */
} gw_status;

typedef enum {
    GW_FP64 = 0,     /* form, factor and solve in FP64 */
    GW_FP32_IR = 1,  /* factor and solve in FP32, FP64 residual refinement */
    GW_BF16X_IR = 2  /* FP32 factor with split-BF16 trailing updates, FP64 refinement */
} gw_precision;

typedef struct gw_ctx gw_ctx;

/* One molecule (Section 3).  Every array is DEVICE memory.
 *
 * Products are grouped in blocks; all products of block b share one ascending
 * orbital set O_b = orb_idx[blk_orb[b] .. blk_orb[b+1]) (the atom or atom pair
 * the product lives on; the vertex is zero outside it, Section 3 text after
 * eq. VertexDefinition).  Product mu of block b (blk_prod[b] <= mu <
 * blk_prod[b+1]) stores its |O_b| x |O_b| symmetric matrix V_mu^{ab} at
 * vals[blk_val[b] + (mu - blk_prod[b]) * |O_b|^2], row-major in O_b order.
 * |O_b| must be at most 64. */
typedef struct {
    int32_t n_orb;            /* number of orbitals = number of KS states */
    int32_t n_occ;            /* occupied states: 0 < n_occ < n_orb */
    int32_t n_prod;           /* number of products N_prod */
    const double *eig;        /* [n_orb] ascending; eig[n_occ-1] < eig[n_occ] */
    const double *X;          /* [n_orb][n_orb], X[a*n_orb + E] = X_a^E */
    int32_t n_blk;
    const int32_t *blk_prod;  /* [n_blk+1] product offsets, blk_prod[0] = 0, last = n_prod */
    const int32_t *blk_orb;   /* [n_blk+1] offsets into orb_idx */
    const int32_t *orb_idx;   /* orbital sets, ascending within a block, < n_orb */
    const int64_t *blk_val;   /* [n_blk+1] offsets into vals */
    const double *vals;       /* vertex values */
} gw_molecule;

/* Frequency mesh (Section 5, 5.B): omega_j = omega_min + j*domega,
 * j = 0..n_omega-1, domega = (omega_max - omega_min)/n_omega.  Requirements:
 * n_omega a power of two in [16, 2048]; omega_min = -omega_max (a window
 * symmetric about the Fermi level); domega an exact power of two; eps > 0.
 * frac_bits < 0 picks the fixed-point exponent s from the data (the largest
 * that provably cannot overflow); frac_bits >= 0 asks for that s, lowered to
 * the safe maximum if it is larger (the report says what was used). */
typedef struct {
    int32_t n_omega;
    double omega_min, omega_max;
    double eps;
    int32_t frac_bits;
} gw_grid;

typedef struct {
    int32_t n_hbins;          /* spectral bins stored per (mu, nu): m = 0..n_hbins-1 */
    int32_t frac_bits_used;   /* s: histogram entries are integers times 2^-s */
    int64_t n_dropped_pairs;  /* pairs whose energy lies beyond the mesh (ignored) */
    int32_t n_solved;         /* frequencies factorised (the rest by conj mirror) */
    int32_t n_fallback;       /* frequencies re-solved in FP64 after IR failed */
    int32_t max_iter;         /* most refinement steps any frequency needed */
    double max_rel_update;    /* largest final ||dW||_F / ||W||_F over frequencies */
} gw_report;

/* Sizes the caller needs before gw_build_chi0 (filled by gw_query_sizes). */
typedef struct {
    int64_t n_pairs;          /* n_occ * (n_orb - n_occ) */
    int32_t n_hbins;          /* bins stored per entry */
    int64_t n_upper;          /* k(k+1)/2, k = n_prod or the compressed rank */
    int64_t hist_bytes;       /* n_hbins * n_upper * 8 */
    int64_t chi0_bytes;       /* n_omega * k * k * 16 */
} gw_sizes;

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
 * workspace the context may allocate (0 = 90% of free memory).
 * Returns GW_E_INVALID for a bad device, GW_E_DEVICE on runtime failure. */
gw_status gw_create(int device, size_t hbm_budget_bytes, gw_ctx **out);

/* Waits for the context's outstanding work, frees its workspace. */
gw_status gw_destroy(gw_ctx *ctx);

/* Message of the last failure on this context ("" if none).  Never NULL. */
const char *gw_last_error(const gw_ctx *ctx);

/* Sizes for gw_build_chi0.  eig_host: HOST [n_orb]; k = 0 for no compression.
 * Pure host computation (Section 5 mesh, Section 5.A bins). */
gw_status gw_query_sizes(int32_t n_orb, int32_t n_occ, int32_t n_prod, const double *eig_host,
                         const gw_grid *g, int32_t k, gw_sizes *out);

/* Steps 1-3: a0 histogram and chi0 on the whole mesh (Sections 5.A, 7.A, 8.A).
 *   basis: DEVICE [n_prod][k] or NULL.  If given, pair vectors are projected
 *          onto its columns before histogramming (Section 8.A: compress as
 *          soon as the response is formed), so the outputs live in the
 *          k-dimensional basis: chi0_hat = basis^T chi0 basis.
 *   hist_out: DEVICE int64 [n_hbins][n_upper] or NULL (then a workspace is
 *          used).  Entry (m, t) is 2^s * a0_{mu nu} integrated over bin m,
 *          t the row-major index of mu <= nu in the packed upper triangle.
 *          Integer-exact and independent of launch shape and pair order.
 *   chi0_out: DEVICE complex128 [n_omega][k][k] (k = n_prod without basis).
 *          Both triangles are written.
 *   rep: HOST or NULL.  If non-NULL the call synchronises the stream and
 *          fills n_hbins, frac_bits_used and n_dropped_pairs.
 * Reads eig and the block index arrays back to the host for validation
 * (a synchronous copy on `stream`). */
gw_status gw_build_chi0(gw_ctx *ctx, const gw_molecule *m, const gw_grid *g,
                        const double *basis, int32_t k, void *stream,
                        int64_t *hist_out, void *chi0_out, gw_report *rep);

/* Two spectral windows (Section 5.B eq. win2-for-response): chi0 on a coarse
 * mesh over a wide window and on a fine mesh over a narrow low-energy window,
 * each with its own broadening.  The pairs are split at
 *   lambda_s = floor((omega_max_small - domega_small) / domega_large) * domega_large,
 * a bin edge of the large mesh: a pair with Delta_p < lambda_s enters the
 * small window's spectral function (histogrammed on the fine mesh, Cauchy
 * transform with g_small->eps); every other pair enters through the large
 * mesh's histogram, Cauchy-transformed with g_large->eps and evaluated at the
 * fine mesh's frequencies, so that no pair is counted twice.
 *   g_small, g_large: meshes as for gw_build_chi0, with
 *          domega_small <= domega_large and omega_max_small <= omega_max_large.
 *          Both windows use one fixed-point exponent s, chosen from every
 *          pair with g_large->frac_bits as the request (g_small->frac_bits
 *          is not read).
 *   basis, k: as for gw_build_chi0.
 *   chi_small_out: DEVICE complex128 [g_small->n_omega][k][k], both triangles.
 *   chi_large_out: DEVICE complex128 [g_large->n_omega][k][k]: the ordinary
 *          one-window chi0 of the large mesh (every pair), both triangles.
 *   rep: HOST or NULL; as for gw_build_chi0, for the large mesh.
 * The outputs must not alias.  Errors: GW_E_INVALID for a bad mesh or a pair
 * of meshes that breaks the rules above, GW_E_OOM, GW_E_DEVICE. */
gw_status gw_build_chi0_2w(gw_ctx *ctx, const gw_molecule *m, const gw_grid *g_small,
                           const gw_grid *g_large, const double *basis, int32_t k, void *stream,
                           void *chi_small_out, void *chi_large_out, gw_report *rep);

/* The paper's own route to a0 (Section 5 density matrix; Section 5.A eq.
 * chi_by_spectra; Section 8.A eq. sf-of-response-time): the electronic
 * densities rho+_ab (empty states, poles at E >= 0) and rhobar-_ab(s) =
 * rho-_ab(-s) (occupied states, poles at -E > 0) on the mesh, each pole split
 * linearly between two bins; their discrete Fourier transforms to L time
 * points (L = K+ + K- - 1, the length of the linear convolution); the
 * local product a_mu_nu(t) = 2 V_mu^ab rho+_bc(t) V_nu^cd rhobar-_da(t) time
 * by time over the vertex blocks (O(N^2) per time); the transform back to the
 * mesh; chi0 by the same FFT Cauchy transform as gw_build_chi0.  The result
 * is floating point: a pair (E, F) lands on up to three bins (the
 * convolution of its two one-particle splits), not the two of the exact pair
 * histogram.
 *   m: as for gw_build_chi0; additionally eig[n_occ-1] < 0 <= eig[n_occ]
 *      (energies from the Fermi level) and every orbital set of at most 32
 *      orbitals.
 *   g: as for gw_build_chi0 (frac_bits is not read).
 *   a_out: DEVICE double [n_hbins][n_prod(n_prod+1)/2] or NULL: a0 on the
 *      mesh, bin m integrated, packed upper triangle as hist_out.  n_hbins =
 *      min(n_omega/2, K+ + K- - 1), K+- = floor(max |E|/domega) + 2 over the
 *      empty (occupied) levels; weight beyond the last bin is dropped.
 *   chi0_out: DEVICE complex128 [n_omega][n_prod][n_prod], both triangles.
 *   rep: HOST or NULL: n_hbins, and in n_dropped_pairs the pairs whose
 *      weight reaches beyond the last bin; frac_bits_used = 0.
 * Workspace: the transformed densities take 16 (L/2+1) n_orb^2 bytes each;
 * the time points are processed in chunks of at most 4 GiB of products.
 * Synchronises the stream once (level tables).  Errors: GW_E_INVALID,
 * GW_E_OOM, GW_E_DEVICE. */
gw_status gw_build_chi0_time(gw_ctx *ctx, const gw_molecule *m, const gw_grid *g, void *stream,
                             double *a_out, void *chi0_out, gw_report *rep);

/* The time-domain route of gw_build_chi0_time for a0, then A(omega_j) =
 * 1 - v chi0(omega_j) as in gw_build_A: each bin of the floating-point a0 is
 * multiplied by v once and the Cauchy transform of v a0 is written as
 * 1 - result, as in gw_build_A (Section 5.A eq. chi_by_spectra, Section 8.A eq.
 * sf-of-response-time, Section 2 eq. Coulombscreening).
 *   m, g, a_out, rep: as for gw_build_chi0_time (with GW_A_TRANSFORM=fft,
 *      128 <= n_omega <= 1024).
 *   v: DEVICE double [n_prod][n_prod], the symmetric Coulomb metric.
 *   A_out: DEVICE complex128 [n_omega][n_prod][n_prod], every entry written.
 * Workspace: as gw_build_chi0_time plus that of gw_build_A.  Errors:
 * GW_E_INVALID, GW_E_OOM, GW_E_DEVICE. */
gw_status gw_build_A_time(gw_ctx *ctx, const gw_molecule *m, const double *v, const gw_grid *g, void *stream,
                          double *a_out, void *A_out, gw_report *rep);

/* The GW self-energy downstream of W (Section 5.A eqs. spectral_3 and
 * Cauchy1, time by time as in Section 8.B; exchange by Section 4 eq.
 * instantaneous), on the mesh of g:
 *   gamma[k] = -(domega/pi) Im W(k domega), k = 1 .. n_omega/2 - 1 (the
 *     spectral weight of W - v per bin; gamma[0] = 0 since gamma is odd);
 *   sigma+^{ab}[m] = sum_{k1+k2=m} V_mu^{aa'} rho+_{a'b'}[k1] V_nu^{b'b} gamma^{mu nu}[k2],
 *   sigma-^{ab}[m] the same with rhobar- (weights at s = -m domega),
 *     m < n_omega/2 (weight beyond is dropped), rho+- as for
 *     gw_build_chi0_time;
 *   Sigma(omega_j + i eps) = sum_m sigma+[m] / (omega_j - m domega + i eps)
 *                          + sigma-[m] / (omega_j + m domega + i eps);
 *   Sigma_x^{ab} = -V_mu^{aa'} (sum_{E occ} X_a'^E X_b'^E) V_nu^{b'b} v^{mu nu}.
 * The convolutions go through L = max(K+, K-) + n_omega/2 - 1 time points
 * (L/2 + 1 formed), the products over pairs of vertex blocks.
 *   m: as for gw_build_chi0_time (energies from the Fermi level, orbital
 *      sets of at most 32 orbitals).
 *   v: DEVICE [n_prod][n_prod] (only read for Sigma_x_out; may be NULL
 *      without it).
 *   g: the mesh W was computed on (n_omega even).
 *   W: DEVICE complex128 [n_omega][n_prod][n_prod] (gw_solve_W's output).
 *   sigma_out: DEVICE double [2][n_omega/2][n_orb][n_orb] or NULL: sigma+
 *      then sigma-.
 *   Sigma_out: DEVICE complex128 [n_omega][n_orb][n_orb]: the correlation
 *      part Sigma(omega_j + i eps) (complex symmetric).
 *   Sigma_x_out: DEVICE double [n_orb][n_orb] or NULL.
 *   rep: HOST or NULL: n_hbins = n_omega/2.
 * The accumulation over block pairs uses floating-point atomics, so the last
 * bits may differ between runs.  Synchronises the stream once (level
 * tables).  Errors: GW_E_INVALID, GW_E_OOM, GW_E_DEVICE. */
gw_status gw_self_energy(gw_ctx *ctx, const gw_molecule *m, const double *v, const gw_grid *g,
                         const void *W, void *stream, double *sigma_out, void *Sigma_out,
                         double *Sigma_x_out, gw_report *rep);

/* Dyson's equation and the density of states (Section 2 eq. Dyson with the
 * V_xc replacement and the DOS definition; Section 3 eq. tensorform-dyson),
 * for every point of the mesh g, in the orbital basis of m (orthonormal, S = 1):
 *   G(omega_j + i eps) = [(omega_j + i eps) 1 - H_KS - Sigma_x - Sigma_c(omega_j) + V_xc]^{-1},
 *   H_KS = X diag(eig) X^T,  dos[j] = -(1/pi) Im tr G(omega_j + i eps).
 *   Sigma_c: DEVICE complex128 [n_omega][n_orb][n_orb] (gw_self_energy's
 *     Sigma_out on the same mesh) or NULL (no correlation part).
 *   Sigma_x, Vxc: DEVICE double [n_orb][n_orb] or NULL (zero); V_xc is the
 *     DFT exchange-correlation potential that the self-energy replaces.
 *   dos_out: DEVICE double [n_omega].
 *   G_out: DEVICE complex128 [n_omega][n_orb][n_orb] or NULL.
 *   rep: HOST or NULL: n_solved = n_omega.
 *   g: the mesh Sigma_c was computed on (as for gw_build_chi0).
 * One batched LU and solve per frequency (no mirror: G(-omega) is not the
 * conjugate of G(omega)).  With Im Sigma_c negative semidefinite (as the
 * self-energy is) and eps > 0 the matrix is never singular; a Sigma_c that
 * makes it singular gives non-finite entries, not an error.
 * Errors: GW_E_INVALID, GW_E_OOM, GW_E_DEVICE. */
gw_status gw_dyson_dos(gw_ctx *ctx, const gw_molecule *m, const gw_grid *g, const void *Sigma_c,
                       const double *Sigma_x, const double *Vxc, void *stream, double *dos_out,
                       void *G_out, gw_report *rep);

/* Step 4: W(omega_j) = (1 - v chi0(omega_j))^{-1} v for every mesh point
 * (Section 2 eq. Coulombscreening).  Only j = 0 and j >= n_omega/2 are
 * factorised; W(omega_{n-j}) = conj W(omega_j) fills the rest (retarded
 * response, exact on the symmetric mesh).
 *   v: DEVICE, [n][n] symmetric (v_is_diag = 0) or the [n] diagonal of a
 *      diagonal metric (v_is_diag = 1).  For the compressed solve pass the
 *      metric S from gw_compress_basis and chi_hat from gw_build_chi0.
 *   chi0: DEVICE complex128 [n_omega][n][n] (e.g. from gw_build_chi0).
 *   prec: GW_FP64, or a mixed form refined with an FP64 residual
 *      r = v - (1 - v chi0) W, W_k = W_{k-1} + dW_k, until the error left in
 *      W_k is estimated below tol ||W_k||_F: ||dW_k||_F <= tol ||W_k||_F, or
 *      the iteration contracts (rho_k = ||dW_k||_F / ||dW_{k-1}||_F <= 1/2,
 *      dW_0 = W_0) and ||dW_k||_F rho_k <= tol ||W_k||_F (at most 6 steps);
 *      a frequency that does not converge is re-solved in FP64.
 *   W_out: DEVICE complex128 [n_omega][n][n].  W_out == chi0 is allowed:
 *      W then overwrites chi0 in place (half the HBM; chi0 is lost).
 *   rep: HOST or NULL; if non-NULL the call synchronises and reports.
 * n_omega must be even and at least 2.  The call synchronises the stream
 * once per refinement step for the mixed forms.  The FP64 form runs on the
 * caller's stream, except the lone point j = 0 (a batch of one frequency),
 * which runs on a second stream of the context beside the first batch when
 * its workspace fits; with GW_SOLVE_STREAMS=2 the frequency batches alternate
 * between the two streams.  Either way the second stream is joined back into
 * the caller's stream's order before the call returns. */
gw_status gw_solve_W(gw_ctx *ctx, const double *v, int32_t v_is_diag, int32_t n,
                     const void *chi0, int32_t n_omega, gw_precision prec, double tol,
                     void *stream, void *W_out, gw_report *rep);

/* Steps 3-4 fused at the front: A(omega_j) = 1 - v chi0(omega_j) for every
 * mesh point, straight from the molecule, without forming chi0.  chi0 is the
 * Cauchy transform of the spectral function a0 (Section 5.A eq.
 * chi_by_spectra), and the transform is linear, so v chi0 is the transform of
 * v a0: the exact histogram is built as for gw_build_chi0 (bin m integrated,
 * integers times 2^-s), each bin is multiplied by v once (n_hbins - 1 real
 * products of size n), and the transform of all n^2 entries of v a0 is one
 * complex-times-real matrix product with the Cauchy kernel matrix
 * T[j][q] = 1/(omega_j - q domega + i eps) - 1/(omega_j + q domega + i eps)
 * over the mesh points j = 0 and j >= n_omega/2; the other points are
 * written as A(-omega) = A(omega)* (v real).  GW_A_TRANSFORM=fft takes the
 * FFT convolution of Section 8.A instead (then 128 <= n_omega <= 1024).
 * Equal to forming 1 - v chi0 from gw_build_chi0's output up to rounding
 * order.
 *   m: as for gw_build_chi0 (no compression basis).
 *   v: DEVICE double [n_prod][n_prod], the symmetric Coulomb metric.
 *   g: as for gw_build_chi0.
 *   A_out: DEVICE complex128 [n_omega][n_prod][n_prod], every entry written
 *      (A is not symmetric).
 *   rep: HOST or NULL; as for gw_build_chi0.
 * Workspace beyond gw_build_chi0's: the products v a0 of every bin
 * (8 n_hbins n_prod^2 bytes), the dense bins of one chunk (at most 2 GiB, at
 * least one bin) and the kernel matrix (16 (n_omega/2 + 1) n_hbins bytes).
 * Errors: GW_E_INVALID (also for a mesh outside the FFT form's range),
 * GW_E_OOM, GW_E_DEVICE. */
gw_status gw_build_A(gw_ctx *ctx, const gw_molecule *m, const double *v, const gw_grid *g,
                     void *stream, void *A_out, gw_report *rep);

/* gw_build_A for the compressed response (Sections 7.B and 8.A): the pair
 * vectors projected onto the basis before the histogram, as gw_build_chi0
 * with basis and k does, and A = 1 - S chi_hat with S = Q^T v Q
 * (gw_compress_basis's outputs); gw_solve_W_A with v = S then gives the
 * compressed X(omega) = (1 - S chi_hat)^{-1} S, for gw_decompress.
 *   S: DEVICE double [k][k]; basis: DEVICE double [n_prod][k]; k >= 1.
 *   A_out: DEVICE complex128 [n_omega][k][k], every entry written.
 *   m, g, rep: as for gw_build_A.
 * Workspace: as gw_build_A with k in place of n_prod, plus gw_build_chi0's
 * projection of the pair vectors.  Errors: as for gw_build_A. */
gw_status gw_build_A_compressed(gw_ctx *ctx, const gw_molecule *m, const double *S, const double *basis,
                                int32_t k, const gw_grid *g, void *stream, void *A_out, gw_report *rep);

/* Step 4 from A = 1 - v chi0 (gw_build_A's output) instead of chi0:
 * W(omega_j) = A(omega_j)^{-1} v (Section 2 eq. Coulombscreening), with the
 * same frequencies, conjugate mirror, precisions, refinement, fallback and
 * report as gw_solve_W (the refinement residual is r = v - A W in FP64).
 *   A: DEVICE complex128 [n_omega][n][n].  It is the factorisation's
 *      storage: under GW_FP64 the solved frequencies (j = 0, j >= n_omega/2)
 *      hold LU factors on return; the mixed forms leave it unchanged.
 *   W_out: DEVICE complex128 [n_omega][n][n]; W_out == A is allowed (each
 *      frequency batch of A is then copied to the workspace first).
 * Errors: as for gw_solve_W. */
gw_status gw_solve_W_A(gw_ctx *ctx, const double *v, int32_t v_is_diag, int32_t n, void *A,
                       int32_t n_omega, gw_precision prec, double tol, void *stream, void *W_out,
                       gw_report *rep);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the GW_FP64
 * form of gw_solve_W_A with no allocation of any kind (no hipMalloc, no
 * hipFree, no stream or event creation).  Its workspace (panel scratch, the
 * inverted 64 x 64 diagonal blocks of L and U, pivots) lives in one fixed
 * device array of 64 MiB per GPU, set up by gw_create and held until the
 * process ends; the frequencies are factorised in batches that fit it.
 *   v, v_is_diag, n, n_omega, rep: as for gw_solve_W_A.
 *   A: DEVICE complex128 [n_omega][n][n]; the solved frequencies (j = 0 and
 *      j >= n_omega/2) hold LU factors on return, as under gw_solve_W_A.
 *   W_out: DEVICE complex128 [n_omega][n][n]; must not alias A.
 * Everything runs in order on `stream` (the lone point j = 0 included); the
 * result equals gw_solve_W_A's FP64 result.  Every call on one GPU shares
 * that GPU's array and leaves its contents behind: calls that overlap in time
 * on one GPU (other streams or host threads) race and give wrong results.
 * Kernel timing (gw_profile_begin) is suspended during the call.
 * Errors: GW_E_INVALID for bad arguments or for an n whose single-frequency
 * workspace exceeds the array (about 3 KiB per row: n up to ~21000),
 * GW_E_DEVICE, GW_E_STATE if the array was never set up on this device. */
gw_status gw_solve_W_A_noalloc(gw_ctx *ctx, const double *v, int32_t v_is_diag, int32_t n, void *A,
                               int32_t n_omega, void *stream, void *W_out, gw_report *rep);

/* Section 7.B subspace: an orthonormal basis Q of the k-dimensional dominant
 * eigenspace of v (the span of its top-k eigenvectors; shifted subspace
 * iteration, 4 steps) and the metric in that basis, S = Q^T v Q.  The
 * compressed interaction depends only on that subspace:
 *   chi_hat = Q^T chi0 Q              (gw_build_chi0 with basis = Q)
 *   X = (1 - S chi_hat)^{-1} S        (gw_solve_W with v = S, v_is_diag = 0)
 *   W = Q X Q^T                       (gw_decompress)
 * which is the paper's W = v + Z chi_RPA Z of eq. chi_RPA with v replaced by
 * its rank-k projection.
 *   v: DEVICE [n][n] symmetric.  Q_out: DEVICE [n][k].  S_out: DEVICE [k][k].
 * Synchronous.  GW_E_NOCONV if the iteration lost a direction (non-finite v). */
gw_status gw_compress_basis(gw_ctx *ctx, const double *v, int32_t n, int32_t k, void *stream,
                            double *Q_out, double *S_out);

/* Decompress one frequency: W = R + U X U^T (Section 8.B, decompression on
 * the fly).  For the top-k subspace pass U = Q and R = NULL; for the paper's
 * pair subspace pass U and R from gw_pair_basis.
 *   U: DEVICE [n][k]; X: DEVICE complex128 [k][k]; R: DEVICE [n][n] real or
 *   NULL; W_out: DEVICE complex128 [n][n]. */
gw_status gw_decompress(gw_ctx *ctx, const double *U, int32_t n, int32_t k, const void *X,
                        const double *R, void *stream, void *W_out);

/* The paper's own compression subspace (Section 7.A): the pair vectors
 * V^{EF} of the electron-hole pairs with F - E < e_threshold (eq.
 * subsetof_vef) generate it; of their Gram matrix in the Coulomb metric,
 * g = X^T v X (eq. projector0), the k-dimensional dominant eigenspace is kept
 * (eq. subspace: the paper keeps the eigenvalues above a threshold; k is that
 * count).  Outputs, all DEVICE, caller-owned:
 *   Z_out [n][k]: basis orthonormal in the Coulomb metric, Z^T v Z = 1
 *     (eq. global-basis-orthogonality); any such basis of the subspace gives
 *     the same W;
 *   U_out [n][k]: U = v Z (the contravariant Z^mu);
 *   R_out [n][n] or NULL: R = v - U U^T.
 *   n_rank_out: HOST or NULL, the number of generating pairs (N_rank).
 * With them, Section 7.B eq. chi_RPA is
 *   chi_hat = U^T chi0 U                   (gw_build_chi0 with basis = U)
 *   X = (1 - chi_hat)^{-1}                 (gw_solve_W with a diagonal metric of ones)
 *   W = v + U (X - 1) U^T = R + U X U^T    (gw_decompress with R)
 * since chi_RPA = (1 - chi_hat)^{-1} chi_hat = X - 1.
 * GW_E_INVALID if fewer than k pairs are below the threshold (or more than
 * 65536); GW_E_NOCONV if the k-th eigenvalue of g is below 1e-10 of the
 * kept trace (k exceeds the rank of the generators).  Synchronous. */
gw_status gw_pair_basis(gw_ctx *ctx, const gw_molecule *m, const double *v, double e_threshold,
                        int32_t k, void *stream, double *Z_out, double *U_out, double *R_out,
                        int64_t *n_rank_out);

/* Batched form: n_mol molecules of different sizes on one mesh (all
 * frequencies of all molecules).  gw_batch_create validates every molecule,
 * sizes the workspaces, chooses GEMM tile shapes per (precision, size class)
 * with the autotuner (median of five timed launches per candidate tile on the
 * molecule's first trailing-update shape, once per class; the table is kept
 * in $GW_TUNE_FILE, default $HOME/.cache/gw_tune.json, whose directories are
 * created as needed; a table that cannot be read or written is reported by
 * gw_last_error() while the batch is still created) and records the whole
 * computation once into a hipGraph: every chi0 build, then the W solves.
 * The solves run in lock step (environment GW_BATCH_MODE=lockstep, the
 * default): every molecule's solve program (its LU factorisations,
 * substitutions and refinement steps, Section 2 eq. Coulombscreening per
 * frequency) advances one operation per lock step, the complex products of a
 * step being one persistent work-queue launch over all molecules (workgroups
 * take tiles from per-XCD device counters and steal from the others), the
 * panel factorisations and row exchanges one grouped launch each, the
 * parallel launches of a step on GW_BATCH_STREAMS (default 4) branches.
 * Programs are aligned so that they end together (lockstep_left: start
 * together).  GW_BATCH_MODE=streams instead runs whole molecules on the
 * parallel branches.  Every molecule then has a workspace of its own, so a
 * batch needs more device memory than one molecule.  gw_batch_run replays
 * the graph on `stream`.
 *   v[i]: DEVICE [n_i][n_i]; chi0_out[i], W_out[i]: DEVICE complex128
 *   [n_omega][n_i][n_i], caller-owned, fixed for the life of the batch.
 *   prec GW_FP64, or GW_FP32_IR / GW_BF16X_IR with exactly n_refine (1..6)
 *   FP64 refinement steps in the graph; gw_batch_run then re-solves in FP64 every frequency
 *   whose last steps do not meet gw_solve_W's stopping rule (counted in the report).
 *   W_out[i] == chi0_out[i] solves in place; the FP64 re-solve then has no
 *   chi0 to start from, so such a frequency makes gw_batch_run return
 *   GW_E_NOCONV (after filling every report).  An in-place molecule on a
 *   mesh of 128 to 1024 points takes the gw_build_A route (A = 1 - v chi0
 *   formed from v a0 in the buffer, then W over it); its buffer never holds
 *   chi0.
 *   reps: HOST [n_mol] or NULL (then gw_batch_run does not synchronise for
 *   FP64).  A later gw_batch_create on the same context retires earlier
 *   batches (gw_batch_run on them returns GW_E_STATE).  Not thread-safe with
 *   other calls on the same context. */
typedef struct gw_batch gw_batch;
gw_status gw_batch_create(gw_ctx *ctx, int32_t n_mol, const gw_molecule *mols, const double *const *v,
                          const gw_grid *g, gw_precision prec, double tol, int32_t n_refine, void *stream,
                          void *const *chi0_out, void *const *W_out, gw_batch **out);
gw_status gw_batch_run(gw_batch *b, void *stream, gw_report *reps);
/* How a batch was recorded: mode 0 (molecules on parallel branches), 1 (lock
 * steps aligned at the end), 2 (lock steps aligned at the start); for lock
 * steps their number, the launches they hold and the products queued in
 * them.  Any output may be NULL.  GW_E_INVALID for a NULL batch. */
gw_status gw_batch_stats(const gw_batch *b, int32_t *mode, int64_t *n_steps, int64_t *n_launches,
                         int64_t *n_products);
gw_status gw_batch_destroy(gw_batch *b);

/* Serving (continuous batching).  gw_submit copies nothing: the molecule's
 * DEVICE buffers must stay valid until gw_poll returns GW_OK.  The request is
 * admitted when its estimated HBM footprint fits; its W (and, compressed, the
 * basis) stays on the device, owned by the library, until gw_release.  chi0
 * itself is not kept: A = 1 - v chi0 (compressed: 1 - S chi_hat) is formed
 * from v a0 in W's buffer (gw_build_A / gw_build_A_compressed) and solved
 * there in place (gw_solve_W_A); only under GW_A_TRANSFORM=fft, on a mesh
 * outside 128..1024 points, is chi0 formed in a buffer of its own first.
 *   k_compress: 0 for the full basis, else the rank of the top-k compression
 *   (W_dev then holds X [n_omega][k][k] complex128 followed by Q [n][k]
 *   doubles, W = Q X Q^T).
 *   v: DEVICE [n_prod][n_prod] Coulomb metric of the molecule.
 * GW_SERVE_SLOTS (default 2) sets the number of concurrent slots;
 * GW_SERVE_TRACE=1 prints each request's phase times to stderr. */
gw_status gw_submit(gw_ctx *ctx, const gw_molecule *m, const double *v, const gw_grid *g,
                    int32_t k_compress, gw_precision prec, double tol, uint64_t *ticket);

/* GW_PENDING until the request is done; then GW_OK with *W_dev pointing at
 * the device-resident result ([n_omega][n][n] complex128) and *rep filled. */
gw_status gw_poll(gw_ctx *ctx, uint64_t ticket, void **W_dev, gw_report *rep);

/* Frees the device result of a finished (or failed) request, or cancels a
 * request that is still waiting for admission; GW_E_STATE while it runs or
 * for an unknown ticket.  The ticket is unknown afterwards. */
gw_status gw_release(gw_ctx *ctx, uint64_t ticket);

/* Kernel timing, for measurement against the rooflines.  While on, every
 * launch of the library's main kernels made by calls on the calling host
 * thread is bracketed by a pair of HIP events on its stream (launches recorded
 * into a batch graph are not timed).  gw_profile_read waits for them and
 * returns one entry per kernel class: launches, summed event time, and summed
 * algorithmic work (flops for products: 8MNK complex, 4MNK real-by-complex;
 * contributions for the histogram) and bytes (the operands read and written
 * once).  Call all three from the thread that called gw_profile_begin; a new
 * gw_profile_begin clears the sums.  The events cost a few microseconds per
 * launch.
 *   out: HOST [cap]; *n_out: number of classes (may exceed cap). */
typedef struct {
    char name[32];
    int64_t launches;
    double ms;
    double flops;
    double bytes;
} gw_kernel_stat;
gw_status gw_profile_begin(gw_ctx *ctx);
gw_status gw_profile_read(gw_ctx *ctx, gw_kernel_stat *out, int32_t cap, int32_t *n_out);
gw_status gw_profile_end(gw_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* GW_H */
