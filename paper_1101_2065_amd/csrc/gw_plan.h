// Private planning layer shared by the single-molecule ABI (gw_abi.cpp) and
// the batched driver (gw_batch.cpp).  A plan validates the arguments (which
// may read small index arrays back to the host) and allocates every buffer;
// enqueueing a plan only launches kernels on a stream, with no host
// synchronisation and no allocation, so it can be recorded into a hipGraph.
#pragma once

#include "../../include/gw.h"
#include "gw_ctx.h"
#include "gw_internal.h"

#include <string>
#include <vector>

namespace gwp {

using gwk::zdbl;
using gwk::zflt;

gw_status fail(gw_ctx *c, gw_status s, const std::string &msg);

// Host-forced faults, for testing the error paths without breaking anything
// on the device: the environment variable GW_FAULT (read once per process)
// set to "oom" makes every workspace allocation fail as out of memory,
// "device" makes every checked runtime call report a device failure (a
// sticky error), "noconv" makes every refinement step report that it did not
// converge.  Unset or anything else: no fault.
enum Fault { FAULT_NONE = 0, FAULT_OOM = 1, FAULT_DEVICE = 2, FAULT_NOCONV = 3 };
Fault fault();
// Grow-only named device buffer of the context.
gw_status ws(gw_ctx *c, const std::string &name, size_t bytes, void **out);
// Free every buffer whose name starts with `prefix` (after the device has
// finished its work; for the private context of a serving slot, in its
// stream's order).
void ws_release(gw_ctx *c, const std::string &prefix);

#define GW_HIP(ctx, call)                                                                                     \
    do {                                                                                                      \
        hipError_t _e = (call);                                                                               \
        if (_e == hipSuccess && gwp::fault() == gwp::FAULT_DEVICE) _e = hipErrorLaunchFailure;               \
        if (_e != hipSuccess)                                                                                 \
            return gwp::fail((ctx), _e == hipErrorOutOfMemory ? GW_E_OOM : GW_E_DEVICE,                       \
                             std::string(#call) + ": " + hipGetErrorString(_e));                             \
    } while (0)

struct BuildPlan {
    gw_molecule m{};
    gw_grid g{};
    const double *basis = nullptr;
    int k = 0;
    int n_orb = 0, n_occ = 0, n_prod = 0, n_virt = 0, rows = 0, nhb = 0, kbits = 0, max_o = 0;
    int echunk = 0, splits = 1, j0 = 0;
    int64_t n_pairs = 0, n_upper = 0;
    double dom = 0;
    double dmax = 0;  // largest pair energy eig[n_orb-1] - eig[0]
    double *P = nullptr, *Pt = nullptr, *bt = nullptr, *Ps = nullptr, *fsort = nullptr;
    int32_t *lo = nullptr, *rowoff = nullptr, *binoff = nullptr, *perm = nullptr, *sdev = nullptr;
    int64_t *stat = nullptr, *H = nullptr;
    uint64_t *vmax = nullptr;
    zdbl *Kt = nullptr, *tw = nullptr;
};

// Validate, size and allocate (buffer names get `prefix`).
gw_status build_plan(gw_ctx *c, const gw_molecule *m, const gw_grid *g, const double *basis, int k, hipStream_t st,
                     const std::string &prefix, int64_t *hist_out, BuildPlan *p);
// Launch a1-a4 for a plan.  with_kspec: also compute the Cauchy-kernel
// spectrum (once per mesh).
gw_status build_enqueue(gw_ctx *c, const BuildPlan &p, hipStream_t st, void *chi0_out, bool with_kspec);

// A = 1 - v chi0 formed from v a0: the products v a0 of every bin (B, bins
// >= 1; row 0 takes the identity), the dense bins of one chunk (D, dchunk
// bins) and the Cauchy-transform matrix T of the solved half of the mesh.
struct ARouteWs {
    double *D = nullptr, *B = nullptr;
    zdbl *T = nullptr;
    int dchunk = 1;
};
// GW_A_TRANSFORM=fft: the A route's transform by FFT convolution (meshes of
// 128 to 1024 points) instead of the matrix product (any mesh).
bool a_transform_fft();
bool a_mesh_ok(int n_omega);
// Workspace of the route for n products, nhb bins and n_omega mesh points
// (named `prefix`aD/aB/aT; grow-only, so a run of calls leaves buffers that
// fit the largest).
gw_status a_route_ws(gw_ctx *c, const std::string &prefix, int n, int nhb, int n_omega, ARouteWs *w);
// a1-a3 as build_enqueue, then A[j] = 1 - v chi0(omega_j) for all j into A_out.
gw_status a_route_enqueue(gw_ctx *c, const BuildPlan &p, hipStream_t st, const double *v, const ARouteWs &w,
                          bool with_kspec, void *A_out);
// The A route's pipeline over the bins: histogram range c adds the pairs
// whose lower bin lies in [lo, hi); then the products v a0 of bins
// [m0, m0 + cnt) (cnt <= dchunk) run, every one of those bins being final
// (bin m takes weight from the pairs of bins m - 1 and m only).  The ranges
// cover [0, nhb - 1) and the bins [1, nhb) each exactly once; about `want`
// ranges.  Empty for nhb <= 1.
struct HistRange {
    int lo, hi, m0, cnt;
};
void hist_ranges(int nhb, int dchunk, int want, std::vector<HistRange> *out);
// The transform of the products B of the bins into A (both forms below).
gw_status a_transform_enqueue(gw_ctx *c, hipStream_t st, int n, int n_omega, int nhb, const ARouteWs &w,
                              const zdbl *Kt, const zdbl *tw, int j0, double domega, double eps, void *A_out);
// A[j] = 1 - v chi0(omega_j) for all j from a spectral array a [nhb][n(n+1)/2]
// already on the mesh (the exact histogram times 2^-s, or a0 in floating
// point: a_i64 or a_f64): the Cauchy transform of the products v a0 as one
// complex-times-real matrix product over the solved half of the mesh
// (omega_j = (j + j0) domega), the rest by the conjugate mirror; with
// GW_A_TRANSFORM=fft instead the FFT convolution with the Cauchy-kernel
// spectrum Kt, tw over all mesh points.
gw_status a_from_bins_enqueue(gw_ctx *c, hipStream_t st, int n, int n_omega, int nhb, const int64_t *a_i64,
                              const int32_t *s_dev, const double *a_f64, const double *v, const ARouteWs &w,
                              const zdbl *Kt, const zdbl *tw, int j0, double domega, double eps, void *A_out);

struct SolveWs {
    zdbl *A = nullptr;
    zflt *A32 = nullptr, *B32 = nullptr;
    zdbl *R = nullptr;
    void *scratch = nullptr;
    void *Li = nullptr, *Ui = nullptr;
    int32_t *ipiv = nullptr, *perm = nullptr, *info = nullptr, *active = nullptr;
    double *norms = nullptr;
};

struct SolvePlan {
    int n = 0, n_omega = 0, nbmax = 0;
    bool mixed = false;
    SolveWs w;
    // [2][n_omega][2]: |dW|^2, |W|^2 of the last refinement step, then of the
    // step before it
    double *final_norms = nullptr;
};

// Refinement stopping rule.  Step k of W_{k} = W_{k-1} + dW_k contracts the
// error by about rho_k = ||dW_k|| / ||dW_{k-1}|| (with dW_0 = W_0, the first
// low-precision solution), so the error left in W_k is about ||dW_k|| rho_k.
// A frequency has converged when ||dW_k|| <= tol ||W_k||, or when the
// iteration contracts (rho_k <= 1/2) and ||dW_k|| rho_k <= tol ||W_k||.
// dn = ||dW_k||, dprev = ||dW_{k-1}|| (||W_0|| for k = 1), wn = ||W_k||.
bool ir_converged(int k, double dn, double dprev, double wn, double tol);

size_t per_freq_bytes(int n, bool mixed);
int solve_batch_max(int n, int n_omega, bool mixed, size_t budget);
// ws_budget: bytes the solve workspace may take (0: the context budget).
gw_status solve_plan(gw_ctx *c, int n, int n_omega, bool mixed, const std::string &prefix, SolvePlan *p,
                     size_t ws_budget = 0);
// Enqueue all solves of one mesh: FP64, or FP32 with exactly fixed_ir FP64
// refinement steps; the last step's norms go to p.final_norms.  No host
// synchronisation.
// Ain: A = 1 - v chi0 given instead of chi0 (chi0 = NULL): each batch is
// factorised in place in Ain, or from a copy when W aliases Ain.  skip_j0:
// the lone point j = 0 is solved elsewhere.
gw_status solve_enqueue_nosync(gw_ctx *c, SolvePlan &p, hipStream_t st, const double *v, int v_is_diag,
                               const zdbl *chi0, zdbl *W, int fixed_ir, zdbl *Ain = nullptr, bool skip_j0 = false);
// The workspace of frequency batch [j0, j0 + nb) for the route above.
gw_status batch_ws(gw_ctx *c, hipStream_t st, const SolveWs &base, zdbl *Ain, const zdbl *W, int64_t nn, int j0,
                   int nb, SolveWs *out);
// One frequency (or a strided run of them) in FP64; chi0 = NULL: w.A already
// holds A.
gw_status solve_batch_fp64(gw_ctx *c, hipStream_t st, int n, const double *v, int v_is_diag, const zdbl *chi0,
                           zdbl *W, int nb, SolveWs &w);

// Lock-step execution of recorded solve programs (batched form).
struct LockStep;
struct LockStepStats {
    int64_t steps = 0, ops = 0, launches = 0, products = 0;
};
// Group the programs' operations into lock steps (operation k of every
// program in step k, or, right_align, aligned so that all programs end in the
// last step), build and upload the descriptor tables.  Host synchronous.
gw_status lockstep_plan(gw_ctx *c, std::vector<std::vector<gwk::RecOp>> progs, bool right_align, LockStep **out);
// Enqueue every lock step on st (parallel launches of a step on the branches,
// joined before the next step; events: 1 + branches.size()).  Recordable.
gw_status lockstep_enqueue(gw_ctx *c, const LockStep &ls, hipStream_t st, const std::vector<hipStream_t> &branches,
                           const std::vector<hipEvent_t> &events);
const LockStepStats &lockstep_stats(const LockStep *ls);
void lockstep_free(LockStep *ls);

// GEMM tile policy for the launches of the calling host thread (autotuner).
void set_thread_gemm_tile(int tile);
// Complex-float GEMMs of the calling host thread on split-BF16 MFMA (BF16x LU);
// returns the previous setting.
bool set_thread_cgemm_bf16x(bool on);
// Scoped form: BF16x on for the lifetime of the guard when `on`.
struct Bf16xScope {
    bool prev;
    explicit Bf16xScope(bool on) : prev(set_thread_cgemm_bf16x(on)) {}
    ~Bf16xScope() { set_thread_cgemm_bf16x(prev); }
};

}  // namespace gwp
