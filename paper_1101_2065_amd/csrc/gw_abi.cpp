// C ABI of libgw.so: argument checks, planning, workspace and launch order.
// Every arithmetic step of the path runs in the HIP kernels of k_exact.hip,
// k_chi0.hip, k_gemm.hip, k_lu.hip and k_compress.hip; this file only
// validates, sizes and sequences.
#include "gw_plan.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

namespace gwk {
hipError_t launch_perm(hipStream_t st, int n, const int32_t *ipiv, int32_t *perm, int batch);
hipError_t launch_init_rhs_perm(hipStream_t st, int n, const double *v, int v_is_diag, const int32_t *perm, zdbl *B,
                                int64_t sB, int batch);
hipError_t launch_dzgemm(hipStream_t st, int M, int N, int K, double alpha, const double *A, int64_t lda, int64_t sA,
                         const zdbl *B, int64_t ldb, int64_t sB, double beta, zdbl *C, int64_t ldc, int64_t sC,
                         int batch);
hipError_t launch_zdgemm(hipStream_t st, int M, int N, int K, double alpha, const zdbl *A, int64_t lda, int64_t sA,
                         const double *B, int64_t ldb, int64_t sB, double beta, zdbl *C, int64_t ldc, int64_t sC,
                         int batch);
hipError_t launch_transpose_d(hipStream_t st, int rows, int cols, const double *src, double *dst);
hipError_t launch_fill_u32(hipStream_t st, uint32_t *p, int64_t n, uint32_t value);
hipError_t launch_rowgather_z2c(hipStream_t st, int n, int nrhs, const int32_t *perm, const zdbl *src, int64_t sS,
                                zflt *dst, int64_t sD, int batch);
hipError_t launch_c2z_set(hipStream_t st, const zflt *d, zdbl *W, int64_t n_per, int batch);
}  // namespace gwk

using gwk::zdbl;
using gwk::zflt;
using gwp::fail;
using gwp::ws;

namespace gwp {

Fault fault() {
    static const Fault f = [] {
        const char *e = std::getenv("GW_FAULT");
        if (!e) return FAULT_NONE;
        const std::string v(e);
        return v == "oom" ? FAULT_OOM : v == "device" ? FAULT_DEVICE : v == "noconv" ? FAULT_NOCONV : FAULT_NONE;
    }();
    return f;
}

gw_status fail(gw_ctx *c, gw_status s, const std::string &msg) {
    if (c) {
        c->err = msg;
        if (s == GW_E_DEVICE) c->sticky = true;
    }
    return s;
}

// Grow-only named device buffers.  Reallocation waits for the device first,
// except in a serving slot's context: that context only ever uses its own
// stream, so its buffers are stream-ordered allocations on it (no device-wide
// synchronisation, memory recycled by the device's pool).
gw_status ws(gw_ctx *c, const std::string &name, size_t bytes, void **out) {
    DevBuf &b = c->bufs[name];
    if (bytes == 0) bytes = 256;
    if (fault() == FAULT_OOM)
        return fail(c, GW_E_OOM, std::string("workspace ") + name + ": cannot allocate " + std::to_string(bytes) +
                                     " bytes (GW_FAULT=oom)");
    if (b.bytes < bytes) {
        if (b.ptr) {
            if (c->own_stream) {
                GW_HIP(c, hipFreeAsync(b.ptr, c->own_stream));
            } else {
                GW_HIP(c, hipDeviceSynchronize());
                GW_HIP(c, hipFree(b.ptr));
            }
            b.ptr = nullptr;
            b.bytes = 0;
        }
        hipError_t e = c->own_stream ? gwk_malloc_async(&b.ptr, bytes, c->own_stream) : hipMalloc(&b.ptr, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            b.ptr = nullptr;
            return fail(c, GW_E_OOM, std::string("workspace ") + name + ": cannot allocate " +
                                         std::to_string(bytes) + " bytes");
        }
        b.bytes = bytes;
    }
    *out = b.ptr;
    return GW_OK;
}

void ws_release(gw_ctx *c, const std::string &prefix) {
    std::vector<std::string> names;
    for (auto &kv : c->bufs)
        if (kv.first.compare(0, prefix.size(), prefix) == 0) names.push_back(kv.first);
    if (names.empty()) return;
    if (!c->own_stream) (void)hipDeviceSynchronize();
    for (auto &nm : names) {
        void *p = c->bufs[nm].ptr;
        if (p) (void)(c->own_stream ? hipFreeAsync(p, c->own_stream) : hipFree(p));
        c->bufs.erase(nm);
    }
}

}  // namespace gwp

namespace {

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

// domega = 2^-k exactly; returns false otherwise
bool shift_bits(double d, int *k) {
    int e = 0;
    const double m = std::frexp(d, &e);
    if (m != 0.5) return false;
    *k = 1 - e;
    return true;
}

gw_status check_grid(gw_ctx *c, const gw_grid *g, int *kbits) {
    if (!g) return fail(c, GW_E_INVALID, "grid is NULL");
    if (!is_pow2(g->n_omega) || g->n_omega < 16 || g->n_omega > 2048)
        return fail(c, GW_E_INVALID, "n_omega must be a power of two in [16, 2048]");
    if (!(g->omega_max > 0.0) || g->omega_min != -g->omega_max)
        return fail(c, GW_E_INVALID, "the mesh must be symmetric: omega_min = -omega_max < 0");
    if (!(g->eps > 0.0) || !std::isfinite(g->eps)) return fail(c, GW_E_INVALID, "eps must be positive");
    const double d = (g->omega_max - g->omega_min) / g->n_omega;
    if (!shift_bits(d, kbits)) return fail(c, GW_E_INVALID, "domega must be an exact power of two");
    return GW_OK;
}

int hist_bins_range(double dmax, int n_omega, int kbits) {
    const double x = std::ldexp(dmax, kbits);
    const long mmax = (long)std::floor(x);
    return (int)std::min<long>(n_omega / 2, mmax + 2);
}

int hist_bins_host(const double *eig, int n_orb, int n_omega, int kbits) {
    return hist_bins_range(eig[n_orb - 1] - eig[0], n_omega, kbits);
}

struct HostMol {
    std::vector<double> eig;
    std::vector<int32_t> blk_prod, blk_orb, orb_idx;
    std::vector<int64_t> blk_val;
    int max_o = 0;
};

gw_status check_molecule(gw_ctx *c, const gw_molecule *m, hipStream_t st, HostMol *h) {
    if (!m) return fail(c, GW_E_INVALID, "molecule is NULL");
    if (m->n_orb < 2 || m->n_occ < 1 || m->n_occ >= m->n_orb)
        return fail(c, GW_E_INVALID, "need 0 < n_occ < n_orb");
    if (m->n_prod < 1 || m->n_blk < 1) return fail(c, GW_E_INVALID, "need n_prod >= 1 and n_blk >= 1");
    if ((int64_t)m->n_occ * (m->n_orb - m->n_occ) > INT32_MAX)
        return fail(c, GW_E_INVALID, "too many electron-hole pairs");
    if (!m->eig || !m->X || !m->blk_prod || !m->blk_orb || !m->orb_idx || !m->blk_val || !m->vals)
        return fail(c, GW_E_INVALID, "NULL array in molecule");
    h->eig.resize(m->n_orb);
    h->blk_prod.resize(m->n_blk + 1);
    h->blk_orb.resize(m->n_blk + 1);
    h->blk_val.resize(m->n_blk + 1);
    GW_HIP(c, hipMemcpyAsync(h->eig.data(), m->eig, sizeof(double) * m->n_orb, hipMemcpyDeviceToHost, st));
    GW_HIP(c, hipMemcpyAsync(h->blk_prod.data(), m->blk_prod, sizeof(int32_t) * (m->n_blk + 1), hipMemcpyDeviceToHost, st));
    GW_HIP(c, hipMemcpyAsync(h->blk_orb.data(), m->blk_orb, sizeof(int32_t) * (m->n_blk + 1), hipMemcpyDeviceToHost, st));
    GW_HIP(c, hipMemcpyAsync(h->blk_val.data(), m->blk_val, sizeof(int64_t) * (m->n_blk + 1), hipMemcpyDeviceToHost, st));
    GW_HIP(c, hipStreamSynchronize(st));
    for (int i = 0; i < m->n_orb; ++i)
        if (!std::isfinite(h->eig[i])) return fail(c, GW_E_INVALID, "non-finite eigenvalue");
    for (int i = 1; i < m->n_orb; ++i)
        if (h->eig[i] < h->eig[i - 1]) return fail(c, GW_E_INVALID, "eigenvalues must be ascending");
    if (!(h->eig[m->n_occ - 1] < h->eig[m->n_occ]))
        return fail(c, GW_E_INVALID, "need a gap: eig[n_occ-1] < eig[n_occ]");
    if (h->blk_prod[0] != 0 || h->blk_prod[m->n_blk] != m->n_prod || h->blk_orb[0] != 0)
        return fail(c, GW_E_INVALID, "block offsets must start at 0 and end at n_prod");
    const int n_idx = h->blk_orb[m->n_blk];
    if (n_idx < 1) return fail(c, GW_E_INVALID, "empty orbital index");
    h->orb_idx.resize(n_idx);
    GW_HIP(c, hipMemcpyAsync(h->orb_idx.data(), m->orb_idx, sizeof(int32_t) * n_idx, hipMemcpyDeviceToHost, st));
    GW_HIP(c, hipStreamSynchronize(st));
    for (int b = 0; b < m->n_blk; ++b) {
        const int np = h->blk_prod[b + 1] - h->blk_prod[b];
        const int no = h->blk_orb[b + 1] - h->blk_orb[b];
        if (np < 1) return fail(c, GW_E_INVALID, "every block needs at least one product");
        if (no < 1 || no > 64) return fail(c, GW_E_INVALID, "orbital set size must be in [1, 64]");
        if (h->blk_val[b] < 0 || h->blk_val[b + 1] - h->blk_val[b] != (int64_t)np * no * no)
            return fail(c, GW_E_INVALID, "blk_val offsets inconsistent with |O|^2 per product");
        for (int i = h->blk_orb[b]; i < h->blk_orb[b + 1]; ++i) {
            if (h->orb_idx[i] < 0 || h->orb_idx[i] >= m->n_orb) return fail(c, GW_E_INVALID, "orbital index out of range");
            if (i > h->blk_orb[b] && h->orb_idx[i] <= h->orb_idx[i - 1])
                return fail(c, GW_E_INVALID, "orbital indices must be strictly ascending in a block");
        }
        h->max_o = std::max(h->max_o, no);
    }
    return GW_OK;
}

hipStream_t as_stream(void *s) { return (hipStream_t)s; }

// The context's second solve stream and its fork/join events (created once).
gw_status aux_stream(gw_ctx *c) {
    if (!c->aux) GW_HIP(c, hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
    if (!c->fork_ev) GW_HIP(c, hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
    if (!c->join_ev) GW_HIP(c, hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming));
    return GW_OK;
}




}  // namespace

namespace gwp {

bool ir_converged(int k, double dn, double dprev, double wn, double tol) {
    if (fault() == FAULT_NOCONV) return false;
    const double w = std::max(wn, 1e-300);
    if (!(dn == dn) || !(wn == wn)) return false;  // NaN: not converged
    if (dn <= tol * w) return true;
    const double rho = dn / std::max(dprev, 1e-300);
    return k >= 1 && rho <= 0.5 && dn * rho <= tol * w;
}

size_t per_freq_bytes(int n, bool mixed) {
    const size_t nn = (size_t)n * n;
    const int nblk = (n + 63) / 64;
    size_t b = nn * 16;                                    // A (FP64)
    b += (size_t)64 * n * 16 + 4096;                       // panel scratch + swap list
    b += 2 * (size_t)nblk * 64 * 64 * 16;                  // L11^-1, U11^-1
    b += 3 * (size_t)n * 4;                                // ipiv, perm
    if (mixed) b += nn * 8 * 2 + nn * 16 + (size_t)64 * n * 8 + 2 * (size_t)nblk * 64 * 64 * 8;
    return b;
}

int solve_batch_max(int n, int n_omega, bool mixed, size_t budget) {
    // at most half the budget and 24 GiB of solve workspace: beyond a few
    // dozen frequencies per batch the GEMMs are already wide enough
    const size_t pf = per_freq_bytes(n, mixed);
    const size_t cap = std::min<size_t>(budget / 2, (size_t)24 << 30);
    int nb = (int)std::max<size_t>(1, std::min<size_t>(cap / pf, 256));
    return std::max(1, std::min(nb, n_omega / 2));
}

gw_status solve_batch_fp64(gw_ctx *c, hipStream_t st, int n, const double *v, int v_is_diag, const zdbl *chi0,
                           zdbl *W, int nb, SolveWs &w) {
    const int64_t nn = (int64_t)n * n;
    if (chi0) GW_HIP(c, gwk::launch_formA(st, n, v, v_is_diag, chi0, nn, w.A, nn, nullptr, 0, nb));
    GW_HIP(c, gwk::launch_fill_u32(st, (uint32_t *)w.info, nb, 0u));
    GW_HIP(c, gwk::getrf_batched<zdbl>(st, n, w.A, nn, w.ipiv, (zdbl *)w.Li, (zdbl *)w.Ui, (zdbl *)w.scratch, w.info, nb));
    GW_HIP(c, gwk::launch_perm(st, n, w.ipiv, w.perm, nb));
    GW_HIP(c, gwk::launch_init_rhs_perm(st, n, v, v_is_diag, w.perm, W, nn, nb));
    // W = (1 - v chi0)^{-1} v is symmetric for symmetric v and chi0: only its
    // lower triangle is solved for, then mirrored
    GW_HIP(c, gwk::getrs_batched<zdbl>(st, n, n, w.A, nn, w.ipiv, (const zdbl *)w.Li, (const zdbl *)w.Ui, W, nn, nb,
                                       true));
    return GW_OK;
}

}  // namespace gwp

namespace {

size_t solve_ws_bytes(int n, int n_omega, bool mixed, size_t budget) {
    return (size_t)gwp::solve_batch_max(n, n_omega, mixed, budget) * gwp::per_freq_bytes(n, mixed) +
           16 * (size_t)n_omega + 4096;
}

// FP32 factor + solve, first solution W = A32^{-1} v (no refinement yet).
gw_status mixed_first_solve(gw_ctx *c, hipStream_t st, int n, const double *v, int v_is_diag, const zdbl *chi0,
                            zdbl *W, int nb, gwp::SolveWs &w) {
    const int64_t nn = (int64_t)n * n;
    if (chi0) GW_HIP(c, gwk::launch_formA(st, n, v, v_is_diag, chi0, nn, w.A, nn, w.A32, nn, nb));
    else GW_HIP(c, gwk::launch_z2c(st, w.A, w.A32, nn * nb));  // A given: its FP32 copy
    GW_HIP(c, gwk::launch_fill_u32(st, (uint32_t *)w.info, nb, 0u));
    GW_HIP(c, gwk::getrf_batched<zflt>(st, n, w.A32, nn, w.ipiv, (zflt *)w.Li, (zflt *)w.Ui, (zflt *)w.scratch, w.info,
                                       nb));
    GW_HIP(c, gwk::launch_perm(st, n, w.ipiv, w.perm, nb));
    GW_HIP(c, gwk::launch_init_rhs(st, n, v, v_is_diag, w.R, nn, nb));
    GW_HIP(c, gwk::launch_rowgather_z2c(st, n, n, w.perm, w.R, nn, w.B32, nn, nb));
    GW_HIP(c, gwk::getrs_batched<zflt>(st, n, n, w.A32, nn, w.ipiv, (const zflt *)w.Li, (const zflt *)w.Ui, w.B32, nn,
                                       nb));
    GW_HIP(c, gwk::launch_c2z_set(st, w.B32, W, nn, nb));
    return GW_OK;
}

// One refinement step: r = v - (1 - v chi0) W in FP64, dW = A32^{-1} r, W += dW
// (active frequencies only, active may be null = all); norms of dW and W.
gw_status mixed_refine_step(gw_ctx *c, hipStream_t st, int n, const double *v, int v_is_diag, zdbl *W, int nb,
                            gwp::SolveWs &w, const int32_t *active, double *norms) {
    const int64_t nn = (int64_t)n * n;
    GW_HIP(c, gwk::launch_residual(st, n, v, v_is_diag, w.A, nn, W, nn, w.R, nn, nb));
    GW_HIP(c, gwk::launch_rowgather_z2c(st, n, n, w.perm, w.R, nn, w.B32, nn, nb));
    GW_HIP(c, gwk::getrs_batched<zflt>(st, n, n, w.A32, nn, w.ipiv, (const zflt *)w.Li, (const zflt *)w.Ui, w.B32,
                                       nn, nb));
    GW_HIP(c, gwk::launch_c2z_add(st, w.B32, W, nn, nb, active));
    GW_HIP(c, gwk::launch_fill_u64(st, (uint64_t *)norms, 2 * nb, 0ull));
    GW_HIP(c, gwk::launch_norms(st, w.B32, W, nn, nb, norms));
    return GW_OK;
}

// Adaptive refinement: after each step the host reads ||dW_k|| and ||W_k|| of
// every frequency and stops it once gwp::ir_converged says its error is below
// tol (see there).
gw_status solve_batch_mixed(gw_ctx *c, hipStream_t st, int n, const double *v, int v_is_diag, const zdbl *chi0,
                            zdbl *W, int nb, double tol, gwp::SolveWs &w, std::vector<int> *conv_iters,
                            std::vector<double> *rel, int max_iter) {
    gw_status s = mixed_first_solve(c, st, n, v, v_is_diag, chi0, W, nb, w);
    if (s != GW_OK) return s;
    std::vector<int32_t> act(nb, 1);
    std::vector<double> hn(2 * nb), prev(nb, 0.0);
    conv_iters->assign(nb, -1);
    rel->assign(nb, 0.0);
    GW_HIP(c, hipMemcpyAsync(w.active, act.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, st));
    for (int it = 1; it <= max_iter; ++it) {
        s = mixed_refine_step(c, st, n, v, v_is_diag, W, nb, w, w.active, w.norms);
        if (s != GW_OK) return s;
        GW_HIP(c, hipMemcpyAsync(hn.data(), w.norms, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, st));
        GW_HIP(c, hipStreamSynchronize(st));
        bool any = false;
        for (int b = 0; b < nb; ++b) {
            if (!act[b]) continue;
            const double dn = std::sqrt(hn[2 * b]), wn = std::sqrt(hn[2 * b + 1]);
            (*rel)[b] = dn / std::max(wn, 1e-300);
            if (gwp::ir_converged(it, dn, it == 1 ? wn : prev[b], wn, tol)) {
                act[b] = 0;
                (*conv_iters)[b] = it;
            } else {
                any = true;
            }
            prev[b] = dn;
        }
        if (!any) break;
        GW_HIP(c, hipMemcpyAsync(w.active, act.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, st));
    }
    return GW_OK;
}

// frequency batches: {0}, then [n/2, n) in equal chunks of at most nbmax
std::vector<std::pair<int, int>> freq_batches(int n_omega, int nbmax) {
    std::vector<std::pair<int, int>> b;
    if (n_omega == 2) return {{0, 2}};
    b.push_back({0, 1});
    const int cnt = n_omega / 2, nbat = (cnt + nbmax - 1) / nbmax;
    for (int i = 0, j = n_omega / 2; i < nbat; ++i) {
        const int sz = cnt / nbat + (i < cnt % nbat ? 1 : 0);
        b.push_back({j, sz});
        j += sz;
    }
    return b;
}

}  // namespace

namespace gwp {

gw_status build_plan(gw_ctx *ctx, const gw_molecule *m, const gw_grid *g, const double *basis, int k, hipStream_t st,
                     const std::string &pre, int64_t *hist_out, BuildPlan *p) {
    int kbits = 0;
    gw_status s = check_grid(ctx, g, &kbits);
    if (s != GW_OK) return s;
    if (!m) return fail(ctx, GW_E_INVALID, "molecule is NULL");
    if (basis && (k < 1 || k > m->n_prod)) return fail(ctx, GW_E_INVALID, "compressed rank k must be in [1, n_prod]");
    if (!basis && k != 0) return fail(ctx, GW_E_INVALID, "k must be 0 without a basis");
    HostMol h;
    s = check_molecule(ctx, m, st, &h);
    if (s != GW_OK) return s;
    p->m = *m;
    p->g = *g;
    p->basis = basis;
    p->k = k;
    p->kbits = kbits;
    p->n_orb = m->n_orb;
    p->n_occ = m->n_occ;
    p->n_prod = m->n_prod;
    p->n_virt = m->n_orb - m->n_occ;
    p->n_pairs = (int64_t)p->n_occ * p->n_virt;
    p->dmax = h.eig[p->n_orb - 1] - h.eig[0];
    p->nhb = hist_bins_range(p->dmax, g->n_omega, kbits);
    p->rows = basis ? k : p->n_prod;
    p->n_upper = (int64_t)p->rows * (p->rows + 1) / 2;
    p->max_o = h.max_o;
    p->dom = (g->omega_max - g->omega_min) / g->n_omega;
    p->j0 = (int)std::lround(g->omega_min / p->dom);
    const int L = 2 * g->n_omega;
    const int64_t n_pairs = p->n_pairs;
    const int n_prod = p->n_prod, rows = p->rows;
    void *q;
#define GW_WS(name, bytes, dst)                                              \
    do {                                                                     \
        if ((s = ws(ctx, pre + name, (bytes), &q)) != GW_OK) return s;       \
        dst = (decltype(dst))q;                                              \
    } while (0)
    if (basis) {
        // Compress as soon as formed (Section 8.A): pair vectors for a range of
        // occupied states at a time, projected onto the basis, so the full
        // N_prod x N_pairs matrix never has to exist.
        const int64_t cap = std::max<int64_t>(1, (int64_t)(2ll << 30) / (8ll * n_prod * p->n_virt));
        p->echunk = (int)std::min<int64_t>(p->n_occ, cap);
        GW_WS("P", sizeof(double) * n_prod * (int64_t)p->echunk * p->n_virt, p->P);
        GW_WS("Pt", sizeof(double) * rows * n_pairs, p->Pt);
        GW_WS("basisT", sizeof(double) * (int64_t)k * n_prod, p->bt);
    } else {
        p->echunk = p->n_occ;
        GW_WS("P", sizeof(double) * n_prod * n_pairs, p->P);
    }
    GW_WS("Ps", sizeof(double) * rows * n_pairs, p->Ps);
    GW_WS("lo", sizeof(int32_t) * p->n_occ * (p->nhb + 1), p->lo);
    GW_WS("rowoff", sizeof(int32_t) * p->n_occ * p->nhb, p->rowoff);
    GW_WS("binoff", sizeof(int32_t) * p->nhb, p->binoff);
    GW_WS("perm", sizeof(int32_t) * n_pairs, p->perm);
    GW_WS("fsort", sizeof(double) * n_pairs, p->fsort);
    GW_WS("stat", 64, p->stat);
    GW_WS("vmax", 64, p->vmax);
    GW_WS("sdev", 64, p->sdev);
    GW_WS("Kt", sizeof(zdbl) * L, p->Kt);
    GW_WS("tw", sizeof(zdbl) * L, p->tw);
    if (hist_out) p->H = hist_out;
    else GW_WS("H", sizeof(int64_t) * p->nhb * p->n_upper, p->H);
#undef GW_WS
    const int ntiles = (rows + 63) / 64;
    const int ntp = ntiles * (ntiles + 1) / 2;
    int splits = std::max(1, std::min(64, (2048 + ntp - 1) / ntp));
    p->splits = std::min(splits, std::max(1, p->nhb - 1));
    return GW_OK;
}

// a1-a3: pair vectors (projected when a basis is given), bins, exact histogram.
gw_status build_hist_enqueue(gw_ctx *ctx, const BuildPlan &p, hipStream_t st, bool with_hist) {
    const gw_molecule *m = &p.m;
    if (p.basis) {
        GW_HIP(ctx, gwk::launch_transpose_d(st, p.n_prod, p.k, p.basis, p.bt));
        for (int e0 = 0; e0 < p.n_occ; e0 += p.echunk) {
            const int ec = std::min(p.echunk, p.n_occ - e0);
            const int64_t cw = (int64_t)ec * p.n_virt;
            GW_HIP(ctx, gwk::launch_pairvec(st, p.n_orb, p.n_occ, p.n_prod, m->n_blk, m->X, m->blk_prod, m->blk_orb,
                                            m->orb_idx, m->blk_val, m->vals, p.max_o, e0, ec, cw, p.P));
            // Pt[:, chunk] = basis^T P_chunk
            GW_HIP(ctx, gwk::launch_dgemm(st, p.k, (int)cw, p.n_prod, 1.0, p.bt, p.n_prod, 0, p.P, cw, 0, 0.0,
                                          p.Pt + (int64_t)e0 * p.n_virt, p.n_pairs, 0, 1));
        }
    } else {
        GW_HIP(ctx, gwk::launch_pairvec(st, p.n_orb, p.n_occ, p.n_prod, m->n_blk, m->X, m->blk_prod, m->blk_orb,
                                        m->orb_idx, m->blk_val, m->vals, p.max_o, 0, p.n_occ, p.n_pairs, p.P));
    }
    const double *Psrc = p.basis ? p.Pt : p.P;
    GW_HIP(ctx, gwk::launch_absmax(st, Psrc, (int64_t)p.rows * p.n_pairs, p.vmax));
    GW_HIP(ctx, gwk::launch_fracbits(st, p.vmax, p.n_pairs, p.g.frac_bits, p.sdev));
    GW_HIP(ctx, gwk::launch_pair_sort(st, p.n_orb, p.n_occ, m->eig, p.kbits, p.nhb, p.lo, p.rowoff, p.binoff, p.perm,
                                      p.fsort, p.stat));
    GW_HIP(ctx, gwk::launch_gather(st, p.rows, p.n_pairs, Psrc, p.perm, p.stat, p.Ps));
    if (with_hist)
        GW_HIP(ctx, gwk::launch_hist(st, p.rows, p.n_pairs, p.Ps, p.fsort, p.binoff, p.stat, p.sdev, p.nhb, p.H,
                                     p.splits));
    return GW_OK;
}

bool a_transform_fft() {
    const char *tr = std::getenv("GW_A_TRANSFORM");
    return tr && std::string(tr) == "fft";
}

bool a_mesh_ok(int n_omega) { return !a_transform_fft() || (n_omega >= 128 && n_omega <= 1024); }

gw_status a_route_ws(gw_ctx *c, const std::string &pre, int n, int nhb, int n_omega, ARouteWs *w) {
    const size_t nn = (size_t)n * n;
    // dense bins staged at most 2 GiB at a time (at least one bin)
    w->dchunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)std::max(1, nhb - 1), ((size_t)2 << 30) / (8 * nn)));
    void *q;
    gw_status s;
    if ((s = ws(c, pre + "aD", 8 * nn * w->dchunk, &q)) != GW_OK) return s;
    w->D = (double *)q;
    if ((s = ws(c, pre + "aB", 8 * nn * std::max(1, nhb), &q)) != GW_OK) return s;
    w->B = (double *)q;
    if ((s = ws(c, pre + "aT", 16 * (size_t)(n_omega / 2 + 1) * std::max(1, nhb), &q)) != GW_OK) return s;
    w->T = (zdbl *)q;
    return GW_OK;
}

gw_status a_from_bins_enqueue(gw_ctx *ctx, hipStream_t st, int n, int n_omega, int nhb, const int64_t *a_i64,
                              const int32_t *s_dev, const double *a_f64, const double *v, const ARouteWs &w,
                              const zdbl *Kt, const zdbl *tw, int j0, double domega, double eps, void *A_out) {
    // v a0 bin by bin (bins 1 .. nhb-1); its Cauchy transform is v chi0
    const int64_t nn = (int64_t)n * n;
    const int64_t n_upper = (int64_t)n * (n + 1) / 2;
    for (int m0 = 1; m0 < nhb; m0 += w.dchunk) {
        const int cnt = std::min(w.dchunk, nhb - m0);
        if (a_i64) GW_HIP(ctx, gwk::launch_expand_bins(st, n, m0, cnt, a_i64, n_upper, s_dev, w.D));
        else GW_HIP(ctx, gwk::launch_expand_bins(st, n, m0, cnt, a_f64, n_upper, w.D));
        GW_HIP(ctx, gwk::launch_dgemm(st, n, n, n, 1.0, v, n, 0, w.D, n, nn, 0.0, w.B + m0 * nn, n, nn, cnt));
    }
    return a_transform_enqueue(ctx, st, n, n_omega, nhb, w, Kt, tw, j0, domega, eps, A_out);
}

gw_status a_transform_enqueue(gw_ctx *ctx, hipStream_t st, int n, int n_omega, int nhb, const ARouteWs &w,
                              const zdbl *Kt, const zdbl *tw, int j0, double domega, double eps, void *A_out) {
    if (a_transform_fft()) GW_HIP(ctx, gwk::launch_fftconv_A(st, n, n_omega, nhb, w.B, Kt, tw, (zdbl *)A_out));
    else GW_HIP(ctx, gwk::launch_cauchy_A(st, n, n_omega, nhb, j0, domega, eps, w.B, w.T, (zdbl *)A_out));
    return GW_OK;
}

void hist_ranges(int nhb, int dchunk, int want, std::vector<HistRange> *out) {
    out->clear();
    if (nhb <= 1) return;
    // bins 1 .. nhb-1 in runs of `step`; range c's histogram adds the pairs of
    // lower bins [m0, m0 + step) (from bin 0 for the first, to the last pair
    // bin nhb - 2 for the last), after which bins [m0, m0 + step) are final
    const int step = std::max(1, std::min(dchunk, (nhb - 1 + want - 1) / std::max(1, want)));
    for (int m0 = 1; m0 < nhb; m0 += step) {
        const int cnt = std::min(step, nhb - m0);
        out->push_back(HistRange{m0 == 1 ? 0 : m0, m0 + cnt >= nhb ? nhb - 1 : m0 + cnt, m0, cnt});
    }
}

gw_status a_route_enqueue(gw_ctx *ctx, const BuildPlan &p, hipStream_t st, const double *v, const ARouteWs &w,
                          bool with_kspec, void *A_out) {
    gw_status s = build_hist_enqueue(ctx, p, st, false);
    if (s != GW_OK) return s;
    if (with_kspec) GW_HIP(ctx, gwk::launch_kspec(st, p.g.n_omega, p.j0, p.dom, p.g.eps, p.Kt, p.tw));
    // The histogram in chunks of bins on the context's second stream, and the
    // products v a0 of each chunk's bins on st as soon as those bins are
    // final (the histogram works on the vector units, the products on the
    // matrix cores, so the two overlap).  Chunk c adds the pairs whose lower
    // bin lies in [lo, hi); bin m receives from the pairs of bins m - 1 and
    // m, so bins [m0, m1) are final once the chunk with hi = m1 is done.  The
    // integer sums do not depend on their order: H is the same bit for bit.
    const int n = p.rows, nhb = p.nhb;
    const int64_t nn = (int64_t)n * n, n_upper = (int64_t)n * (n + 1) / 2;
    // GW_HIST_CHUNKS ranges (default 4), each at most the staging buffer's bins
    int want = 4;
    if (const char *e = std::getenv("GW_HIST_CHUNKS")) want = std::max(1, std::min(64, std::atoi(e)));
    std::vector<HistRange> rg;
    hist_ranges(nhb, w.dchunk, want, &rg);
    const int nch = (int)rg.size();
    if ((s = aux_stream(ctx)) != GW_OK) return s;
    while ((int)ctx->chunk_ev.size() < nch) {
        hipEvent_t e;
        GW_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->chunk_ev.push_back(e);
    }
    GW_HIP(ctx, gwk::launch_fill_u64(st, (uint64_t *)p.H, (int64_t)nhb * n_upper, 0ull));
    GW_HIP(ctx, hipEventRecord(ctx->fork_ev, st));
    GW_HIP(ctx, hipStreamWaitEvent(ctx->aux, ctx->fork_ev, 0));
    for (int c = 0; c < nch; ++c) {
        GW_HIP(ctx, gwk::launch_hist(ctx->aux, n, p.n_pairs, p.Ps, p.fsort, p.binoff, p.stat, p.sdev, nhb, p.H,
                                     p.splits, rg[c].lo, rg[c].hi, false));
        GW_HIP(ctx, hipEventRecord(ctx->chunk_ev[c], ctx->aux));
    }
    for (int c = 0; c < nch; ++c) {
        const int m0 = rg[c].m0, cnt = rg[c].cnt;
        GW_HIP(ctx, hipStreamWaitEvent(st, ctx->chunk_ev[c], 0));
        GW_HIP(ctx, gwk::launch_expand_bins(st, n, m0, cnt, p.H, n_upper, p.sdev, w.D));
        GW_HIP(ctx, gwk::launch_dgemm(st, n, n, n, 1.0, v, n, 0, w.D, n, nn, 0.0, w.B + m0 * nn, n, nn, cnt));
    }
    // st has waited for the last chunk: the second stream is joined
    return a_transform_enqueue(ctx, st, n, p.g.n_omega, nhb, w, p.Kt, p.tw, p.j0, p.dom, p.g.eps, A_out);
}

gw_status build_enqueue(gw_ctx *ctx, const BuildPlan &p, hipStream_t st, void *chi0_out, bool with_kspec) {
    gw_status s = build_hist_enqueue(ctx, p, st, true);
    if (s != GW_OK) return s;
    if (with_kspec) GW_HIP(ctx, gwk::launch_kspec(st, p.g.n_omega, p.j0, p.dom, p.g.eps, p.Kt, p.tw));
    GW_HIP(ctx, gwk::launch_fftconv(st, p.rows, p.g.n_omega, p.nhb, p.H, p.sdev, p.Kt, p.tw, (zdbl *)chi0_out));
    return GW_OK;
}

gw_status solve_plan(gw_ctx *ctx, int n, int n_omega, bool mixed, const std::string &pre, SolvePlan *p,
                     size_t ws_budget) {
    const int64_t nn = (int64_t)n * n;
    const int nblk = (n + 63) / 64;
    const int nbmax = solve_batch_max(n, n_omega, mixed, ws_budget ? ws_budget : ctx->budget);
    p->n = n;
    p->n_omega = n_omega;
    p->nbmax = nbmax;
    p->mixed = mixed;
    SolveWs &w = p->w;
    gw_status s;
    void *q;
    if ((s = ws(ctx, pre + "sA", (size_t)nbmax * nn * 16, &q)) != GW_OK) return s;
    w.A = (zdbl *)q;
    if ((s = ws(ctx, pre + "sScr", (size_t)nbmax * (64 * (size_t)n * 16 + 4 * 257 + 256), &q)) != GW_OK) return s;
    w.scratch = q;
    const size_t esz = mixed ? 8 : 16;
    if ((s = ws(ctx, pre + "sLi", (size_t)nbmax * nblk * 64 * 64 * esz, &q)) != GW_OK) return s;
    w.Li = q;
    if ((s = ws(ctx, pre + "sUi", (size_t)nbmax * nblk * 64 * 64 * esz, &q)) != GW_OK) return s;
    w.Ui = q;
    if ((s = ws(ctx, pre + "sIpiv", (size_t)nbmax * n * 4, &q)) != GW_OK) return s;
    w.ipiv = (int32_t *)q;
    if ((s = ws(ctx, pre + "sPerm", (size_t)nbmax * n * 4, &q)) != GW_OK) return s;
    w.perm = (int32_t *)q;
    if ((s = ws(ctx, pre + "sInfo", (size_t)nbmax * 4, &q)) != GW_OK) return s;
    w.info = (int32_t *)q;
    if ((s = ws(ctx, pre + "sAct", (size_t)nbmax * 4, &q)) != GW_OK) return s;
    w.active = (int32_t *)q;
    if ((s = ws(ctx, pre + "sNorm", (size_t)nbmax * 16, &q)) != GW_OK) return s;
    w.norms = (double *)q;
    if ((s = ws(ctx, pre + "sFinal", (size_t)n_omega * 32, &q)) != GW_OK) return s;
    p->final_norms = (double *)q;
    if (mixed) {
        if ((s = ws(ctx, pre + "sA32", (size_t)nbmax * nn * 8, &q)) != GW_OK) return s;
        w.A32 = (zflt *)q;
        if ((s = ws(ctx, pre + "sB32", (size_t)nbmax * nn * 8, &q)) != GW_OK) return s;
        w.B32 = (zflt *)q;
        if ((s = ws(ctx, pre + "sR", (size_t)nbmax * nn * 16, &q)) != GW_OK) return s;
        w.R = (zdbl *)q;
    }
    return GW_OK;
}

gw_status batch_ws(gw_ctx *c, hipStream_t st, const SolveWs &base, zdbl *Ain, const zdbl *W, int64_t nn, int j0,
                   int nb, SolveWs *out) {
    *out = base;
    if (!Ain) return GW_OK;
    if (Ain == W) GW_HIP(c, gwk::launch_copy(st, out->A, Ain + j0 * nn, sizeof(zdbl) * nn * nb));
    else out->A = Ain + j0 * nn;
    return GW_OK;
}

gw_status solve_enqueue_nosync(gw_ctx *ctx, SolvePlan &p, hipStream_t st, const double *v, int v_is_diag,
                               const zdbl *chi0, zdbl *W, int fixed_ir, zdbl *Ain, bool skip_j0) {
    const int64_t nn = (int64_t)p.n * p.n;
    gw_status s;
    for (auto &bt : freq_batches(p.n_omega, p.nbmax)) {
        const int j0 = bt.first, nb = bt.second;
        if (skip_j0 && j0 == 0 && nb == 1) continue;
        const zdbl *X = chi0 ? chi0 + j0 * nn : nullptr;
        SolveWs w;
        if ((s = batch_ws(ctx, st, p.w, Ain, W, nn, j0, nb, &w)) != GW_OK) return s;
        if (!p.mixed) {
            s = solve_batch_fp64(ctx, st, p.n, v, v_is_diag, X, W + j0 * nn, nb, w);
            if (s != GW_OK) return s;
        } else {
            s = mixed_first_solve(ctx, st, p.n, v, v_is_diag, X, W + j0 * nn, nb, w);
            if (s != GW_OK) return s;
            for (int it = 0; it < fixed_ir; ++it) {
                // the last step's norms go to the first half, the step
                // before it to the second (the stopping rule needs both)
                double *nrm = p.final_norms + 2 * j0 + (it == fixed_ir - 1 ? 0 : 2 * (int64_t)p.n_omega);
                s = mixed_refine_step(ctx, st, p.n, v, v_is_diag, W + j0 * nn, nb, w, nullptr, nrm);
                if (s != GW_OK) return s;
            }
        }
    }
    if (p.n_omega >= 4) GW_HIP(ctx, gwk::launch_conj_mirror(st, nn, p.n_omega, W));
    return GW_OK;
}

}  // namespace gwp

extern "C" {
gw_status gw_create(int device, size_t hbm_budget_bytes, gw_ctx **out) {
    if (!out) return GW_E_INVALID;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return GW_E_DEVICE;
    if (device < 0 || device >= count) return GW_E_INVALID;
    if (hipSetDevice(device) != hipSuccess) return GW_E_DEVICE;
    gwk_noalloc_init(device);
    gw_ctx *c = new gw_ctx();
    c->device = device;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        delete c;
        return GW_E_DEVICE;
    }
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)fr);
    *out = c;
    return GW_OK;
}

gw_status gw_destroy(gw_ctx *ctx) {
    if (!ctx) return GW_E_INVALID;
    gwk_serve_stop(ctx);
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    gwk_prof_release(ctx);
    if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
    for (hipEvent_t e : ctx->chunk_ev) (void)hipEventDestroy(e);
    for (auto &kv : ctx->bufs)
        if (kv.second.ptr) {
            if (ctx->own_stream) (void)hipFreeAsync(kv.second.ptr, ctx->own_stream);
            else (void)hipFree(kv.second.ptr);
        }
    if (ctx->own_stream) (void)hipStreamSynchronize(ctx->own_stream);
    delete ctx;
    return GW_OK;
}

const char *gw_last_error(const gw_ctx *ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

gw_status gw_query_sizes(int32_t n_orb, int32_t n_occ, int32_t n_prod, const double *eig_host, const gw_grid *g,
                         int32_t k, gw_sizes *out) {
    if (!out || !eig_host || n_orb < 2 || n_occ < 1 || n_occ >= n_orb || n_prod < 1 || k < 0 || k > n_prod)
        return GW_E_INVALID;
    int kbits = 0;
    if (check_grid(nullptr, g, &kbits) != GW_OK) return GW_E_INVALID;
    const int64_t kk = k ? k : n_prod;
    out->n_pairs = (int64_t)n_occ * (n_orb - n_occ);
    out->n_hbins = hist_bins_host(eig_host, n_orb, g->n_omega, kbits);
    out->n_upper = kk * (kk + 1) / 2;
    out->hist_bytes = (int64_t)out->n_hbins * out->n_upper * 8;
    out->chi0_bytes = (int64_t)g->n_omega * kk * kk * 16;
    return GW_OK;
}

gw_status gw_build_chi0(gw_ctx *ctx, const gw_molecule *m, const gw_grid *g, const double *basis, int32_t k,
                        void *stream, int64_t *hist_out, void *chi0_out, gw_report *rep) {
    if (!ctx) return GW_E_INVALID;
    if (ctx->sticky) return fail(ctx, GW_E_DEVICE, "context has a sticky device error: " + ctx->err);
    GW_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = as_stream(stream);
    if (!chi0_out) return fail(ctx, GW_E_INVALID, "chi0_out is NULL");
    gwp::BuildPlan p;
    gw_status s = gwp::build_plan(ctx, m, g, basis, k, st, "", hist_out, &p);
    if (s != GW_OK) return s;
    const bool kspec = ctx->ks_n != g->n_omega || ctx->ks_min != g->omega_min || ctx->ks_d != p.dom ||
                       ctx->ks_eps != g->eps;
    s = gwp::build_enqueue(ctx, p, st, chi0_out, kspec);
    if (s != GW_OK) return s;
    if (kspec) {
        ctx->ks_n = g->n_omega;
        ctx->ks_min = g->omega_min;
        ctx->ks_d = p.dom;
        ctx->ks_eps = g->eps;
    }
    if (rep) {
        int64_t hs[2];
        int32_t sv = 0;
        GW_HIP(ctx, hipMemcpyAsync(hs, p.stat, sizeof(hs), hipMemcpyDeviceToHost, st));
        GW_HIP(ctx, hipMemcpyAsync(&sv, p.sdev, sizeof(sv), hipMemcpyDeviceToHost, st));
        GW_HIP(ctx, hipStreamSynchronize(st));
        std::memset(rep, 0, sizeof(*rep));
        rep->n_hbins = p.nhb;
        rep->frac_bits_used = sv;
        rep->n_dropped_pairs = hs[1];
    }
    return GW_OK;
}

gw_status gw_build_chi0_2w(gw_ctx *ctx, const gw_molecule *m, const gw_grid *g_small, const gw_grid *g_large,
                           const double *basis, int32_t k, void *stream, void *chi_small_out, void *chi_large_out,
                           gw_report *rep) {
    if (!ctx) return GW_E_INVALID;
    if (ctx->sticky) return fail(ctx, GW_E_DEVICE, "context has a sticky device error: " + ctx->err);
    GW_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = as_stream(stream);
    if (!chi_small_out || !chi_large_out) return fail(ctx, GW_E_INVALID, "chi_small_out and chi_large_out must be set");
    if (chi_small_out == chi_large_out) return fail(ctx, GW_E_INVALID, "the two outputs must not alias");
    int kbits_s = 0;
    gw_status s = check_grid(ctx, g_small, &kbits_s);
    if (s != GW_OK) return s;
    gwp::BuildPlan pl;
    s = gwp::build_plan(ctx, m, g_large, basis, k, st, "", nullptr, &pl);
    if (s != GW_OK) return s;
    const double ds = (g_small->omega_max - g_small->omega_min) / g_small->n_omega;
    const double dl = pl.dom;
    if (ds > dl) return fail(ctx, GW_E_INVALID, "the small window's spacing must not exceed the large one's");
    if (g_small->omega_max > g_large->omega_max)
        return fail(ctx, GW_E_INVALID, "the small window must lie inside the large one");
    // split energy lambda_s = m_lam * dl: the largest large-mesh bin edge with
    // lambda_s + ds <= omega_max of the small window (powers of two: exact)
    const int m_lam = std::max(0, (int)std::floor((g_small->omega_max - ds) / dl));
    const int ratio = (int)std::lround(dl / ds);
    const int m_cut = m_lam * ratio;  // the same edge on the small mesh
    const int n_s = g_small->n_omega;
    const int nhb_s = hist_bins_range(pl.dmax, n_s, kbits_s);
    const int nh_s = std::min(m_cut, nhb_s - 1) + 1;  // rows of the small histogram that can be non-zero
    const int64_t nu = pl.n_upper;
    const int rows = pl.rows;
    const int L_s = 2 * n_s;
    const int M = pl.nhb - m_lam;  // large-mesh rows that enter the small window's frequencies
    void *q;
    int32_t *lo_s, *rowoff_s, *binoff_s, *perm_s;
    double *fsort_s;
    int64_t *stat_s, *H_s, *Hb = nullptr;
    zdbl *Kt_s, *tw_s, *K = nullptr;
#define GW_WS(name, bytes, dst)                                   \
    do {                                                          \
        if ((s = ws(ctx, name, (bytes), &q)) != GW_OK) return s;  \
        dst = (decltype(dst))q;                                   \
    } while (0)
    GW_WS("2w_lo", sizeof(int32_t) * pl.n_occ * (nhb_s + 1), lo_s);
    GW_WS("2w_rowoff", sizeof(int32_t) * pl.n_occ * nhb_s, rowoff_s);
    GW_WS("2w_binoff", sizeof(int32_t) * nhb_s, binoff_s);
    GW_WS("2w_perm", sizeof(int32_t) * pl.n_pairs, perm_s);
    GW_WS("2w_fsort", sizeof(double) * pl.n_pairs, fsort_s);
    GW_WS("2w_stat", 64, stat_s);
    GW_WS("2w_H", sizeof(int64_t) * nh_s * nu, H_s);
    GW_WS("2w_Kt", sizeof(zdbl) * L_s, Kt_s);
    GW_WS("2w_tw", sizeof(zdbl) * L_s, tw_s);
    if (M > 0) {
        GW_WS("2w_K", sizeof(zdbl) * n_s * M, K);
        if (m_lam > 0) GW_WS("2w_Hb", sizeof(int64_t) * (m_lam + 1) * nu, Hb);
    }
#undef GW_WS
    // large window: the ordinary build over every pair
    const bool kspec = ctx->ks_n != g_large->n_omega || ctx->ks_min != g_large->omega_min || ctx->ks_d != pl.dom ||
                       ctx->ks_eps != g_large->eps;
    s = gwp::build_enqueue(ctx, pl, st, chi_large_out, kspec);
    if (s != GW_OK) return s;
    if (kspec) {
        ctx->ks_n = g_large->n_omega;
        ctx->ks_min = g_large->omega_min;
        ctx->ks_d = pl.dom;
        ctx->ks_eps = g_large->eps;
    }
    // large-mesh histogram of the pairs with Delta >= lambda_s: rows above
    // m_lam are those of the whole histogram; row m_lam loses the upper split
    // weight of the pairs in bin m_lam - 1
    const int64_t *H_lo = nullptr;
    if (M > 0 && m_lam > 0) {
        GW_HIP(ctx, gwk::launch_hist(st, rows, pl.n_pairs, pl.Ps, pl.fsort, pl.binoff, pl.stat, pl.sdev, pl.nhb, Hb,
                                     pl.splits, 0, m_lam));
        int64_t *row = Hb + (int64_t)m_lam * nu;
        GW_HIP(ctx, gwk::launch_sub_i64(st, pl.H + (int64_t)m_lam * nu, row, nu));
        H_lo = row;
    }
    // small window: the pairs with Delta < lambda_s on the fine mesh, same s
    const double *Psrc = pl.basis ? pl.Pt : pl.P;
    GW_HIP(ctx, gwk::launch_pair_sort(st, pl.n_orb, pl.n_occ, pl.m.eig, kbits_s, nhb_s, lo_s, rowoff_s, binoff_s,
                                      perm_s, fsort_s, stat_s));
    GW_HIP(ctx, gwk::launch_gather(st, rows, pl.n_pairs, Psrc, perm_s, stat_s, pl.Ps));
    GW_HIP(ctx, gwk::launch_hist(st, rows, pl.n_pairs, pl.Ps, fsort_s, binoff_s, stat_s, pl.sdev, nhb_s, H_s,
                                 std::min(pl.splits, std::max(1, nhb_s - 1)), 0, m_cut));
    GW_HIP(ctx, gwk::launch_kspec(st, n_s, (int)std::lround(g_small->omega_min / ds), ds, g_small->eps, Kt_s, tw_s));
    GW_HIP(ctx, gwk::launch_fftconv(st, rows, n_s, nh_s, H_s, pl.sdev, Kt_s, tw_s, (zdbl *)chi_small_out, false));
    // the rest, broadened with the large window's eps, at the small mesh's frequencies
    if (M > 0) {
        GW_HIP(ctx, gwk::launch_cauchy_table(st, n_s, g_small->omega_min, ds, pl.nhb, m_lam, dl, g_large->eps, K));
        GW_HIP(ctx, gwk::launch_cauchy_add(st, rows, n_s, pl.nhb, m_lam, pl.H, H_lo, pl.sdev, K,
                                           (zdbl *)chi_small_out));
    }
    GW_HIP(ctx, gwk::launch_symmetrize(st, rows, n_s, (zdbl *)chi_small_out));
    if (rep) {
        int64_t hs[2];
        int32_t sv = 0;
        GW_HIP(ctx, hipMemcpyAsync(hs, pl.stat, sizeof(hs), hipMemcpyDeviceToHost, st));
        GW_HIP(ctx, hipMemcpyAsync(&sv, pl.sdev, sizeof(sv), hipMemcpyDeviceToHost, st));
        GW_HIP(ctx, hipStreamSynchronize(st));
        std::memset(rep, 0, sizeof(*rep));
        rep->n_hbins = pl.nhb;
        rep->frac_bits_used = sv;
        rep->n_dropped_pairs = hs[1];
    }
    return GW_OK;
}

namespace {

// One-particle poles on the mesh, listed bin by bin: the empty states by rising
// energy (bins of E), then the occupied ones by rising -E (bins of -E); each
// level's weight is split between its bin k and k + 1.  Kp, Km: bins of the two
// densities, at most kcap (levels whose weight lies wholly beyond are left out).
struct LevelTables {
    std::vector<int32_t> lev, kb, start;  // start: [Kp + 1] then [Km + 1]
    std::vector<double> ph;
    int nv = 0, Kp = 0, Km = 0;
};

gw_status level_tables(gw_ctx *ctx, const HostMol &h, int n_orb, int n_occ, int kbits, int kcap, LevelTables *t) {
    if (!(h.eig[n_occ - 1] < 0.0 && h.eig[n_occ] >= 0.0))
        return fail(ctx, GW_E_INVALID, "energies must be measured from the Fermi level: eig[n_occ-1] < 0 <= eig[n_occ]");
    const int nv = n_orb - n_occ;
    t->lev.resize(n_orb);
    t->kb.resize(n_orb);
    t->ph.resize(n_orb);
    for (int i = 0; i < n_orb; ++i) {
        const int st_i = i < nv ? n_occ + i : n_occ - 1 - (i - nv);
        const double x = std::ldexp(std::fabs(h.eig[st_i]), kbits);
        const double k = std::floor(x);
        if (!(k < 1e8)) return fail(ctx, GW_E_INVALID, "a level lies too far from the Fermi level for this mesh");
        t->lev[i] = st_i;
        t->kb[i] = (int32_t)k;
        t->ph[i] = x - k;
    }
    t->nv = nv;
    t->Kp = std::min(kcap, t->kb[nv - 1] + 2);
    t->Km = std::min(kcap, t->kb[n_orb - 1] + 2);
    t->start.assign(t->Kp + 1 + t->Km + 1, 0);
    for (int k = 0, i = 0; k <= t->Kp; ++k) {
        while (i < nv && t->kb[i] < k) ++i;
        t->start[k] = i;
    }
    for (int k = 0, i = 0; k <= t->Km; ++k) {
        while (i < n_occ && t->kb[nv + i] < k) ++i;
        t->start[t->Kp + 1 + k] = i;
    }
    return GW_OK;
}

// Vertex block pairs B1 <= B2 (pb1 then pb2 in one array), grouped by tile
// class 2 (|O1| > 16) + (|O2| > 16) with class c at class_off[c] ..
// class_off[c+1] - 1 (class_off may be null), and the largest
// (products x |O|^2) of a block.
int block_pairs(const HostMol &h, int nblk, std::vector<int32_t> *pbs, int *max_vblock, int *class_off = nullptr) {
    std::vector<int32_t> b1s[4], b2s[4];
    for (int b1 = 0; b1 < nblk; ++b1)
        for (int b2 = b1; b2 < nblk; ++b2) {
            const int c = 2 * (h.blk_orb[b1 + 1] - h.blk_orb[b1] > 16) + (h.blk_orb[b2 + 1] - h.blk_orb[b2] > 16);
            b1s[c].push_back(b1);
            b2s[c].push_back(b2);
        }
    pbs->clear();
    int off[5] = {0, 0, 0, 0, 0};
    for (int c = 0; c < 4; ++c) {
        pbs->insert(pbs->end(), b1s[c].begin(), b1s[c].end());
        off[c + 1] = off[c] + (int)b1s[c].size();
    }
    for (int c = 0; c < 4; ++c) pbs->insert(pbs->end(), b2s[c].begin(), b2s[c].end());
    const int npb = off[4];
    if (class_off)
        for (int c = 0; c < 5; ++c) class_off[c] = off[c];
    *max_vblock = 0;
    for (int b = 0; b < nblk; ++b) {
        const int no = h.blk_orb[b + 1] - h.blk_orb[b];
        *max_vblock = std::max(*max_vblock, (h.blk_prod[b + 1] - h.blk_prod[b]) * no * no);
    }
    return npb;
}

}  // namespace

// The time-domain route to a0, then chi0 (v = NULL) or A = 1 - v chi0 formed
// from v a0 (v given) into out.
static gw_status build_time_impl(gw_ctx *ctx, const gw_molecule *m, const double *v, const gw_grid *g, void *stream,
                                 double *a_out, void *chi0_out, gw_report *rep) {
    if (!ctx) return GW_E_INVALID;
    if (ctx->sticky) return fail(ctx, GW_E_DEVICE, "context has a sticky device error: " + ctx->err);
    GW_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = as_stream(stream);
    if (!chi0_out) return fail(ctx, GW_E_INVALID, "the output array is NULL");
    int kbits = 0;
    gw_status s = check_grid(ctx, g, &kbits);
    if (s != GW_OK) return s;
    if (v && !gwp::a_mesh_ok(g->n_omega))
        return fail(ctx, GW_E_INVALID, "gw_build_A_time with GW_A_TRANSFORM=fft needs n_omega in [128, 1024]");
    HostMol h;
    s = check_molecule(ctx, m, st, &h);
    if (s != GW_OK) return s;
    const int n_orb = m->n_orb, n_occ = m->n_occ, n = m->n_prod, nblk = m->n_blk;
    if (h.max_o > TIME_MAX_ORB)
        return fail(ctx, GW_E_INVALID, "the time-domain route takes orbital sets of at most " +
                                           std::to_string(TIME_MAX_ORB) + " orbitals");
    LevelTables lt;
    s = level_tables(ctx, h, n_orb, n_occ, kbits, 1 << 30, &lt);
    if (s != GW_OK) return s;
    const std::vector<int32_t> &lev = lt.lev, &kb = lt.kb, &start = lt.start;
    const std::vector<double> &ph = lt.ph;
    const int nv = lt.nv, Kp = lt.Kp, Km = lt.Km;
    const int nhb = std::min(g->n_omega / 2, Kp + Km - 1);
    // L = the length of the linear convolution: the cyclic one of that length
    // has no wrap-around (the transforms are explicit, any L will do)
    const int L = std::max(2, Kp + Km - 1);
    if (L > (1 << 16)) return fail(ctx, GW_E_INVALID, "the levels span too many mesh points for the time route");
    const int Q = L / 2 + 1;
    // pairs whose convolved weight reaches a bin beyond the mesh
    int64_t dropped = 0;
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < n_occ; ++j) {
            const int top = kb[i] + kb[nv + j] + (ph[i] > 0.0) + (ph[nv + j] > 0.0);
            if (top >= nhb) ++dropped;
        }
    // block pairs B1 <= B2 and the contraction's flop count
    std::vector<int32_t> pbs;
    double cflops = 0.0;
    int max_vblock = 0;
    int class_off[5];
    const int npb = block_pairs(h, nblk, &pbs, &max_vblock, class_off);
    for (int b1 = 0; b1 < nblk; ++b1)
        for (int b2 = b1; b2 < nblk; ++b2) {
            const double n1 = h.blk_orb[b1 + 1] - h.blk_orb[b1], n2 = h.blk_orb[b2 + 1] - h.blk_orb[b2];
            const double pm = h.blk_prod[b1 + 1] - h.blk_prod[b1], pn = h.blk_prod[b2 + 1] - h.blk_prod[b2];
            const double pmn = b1 == b2 ? pm * (pm + 1) / 2 : pm * pn;
            cflops += pn * (4.0 * n1 * n2 * n2 + 8.0 * n1 * n1 * n2) + 4.0 * pmn * n1 * n1;
        }
    const int64_t nn = (int64_t)n_orb * n_orb;
    const int64_t n_upper = (int64_t)n * (n + 1) / 2;
    // time points per chunk: the transformed product of a chunk takes at most 4 GiB
    const int qc = (int)std::max<int64_t>(1, std::min<int64_t>(Q, (int64_t)(4ll << 30) / (16 * n_upper)));
    void *q;
    int32_t *d_lev, *d_start, *d_pb;
    double *d_ph, *rho, *F, *G, *Rp, *Rm, *Ahat, *a = a_out;
    zdbl *Kt, *tw;
#define GW_WS(name, bytes, dst)                                   \
    do {                                                          \
        if ((s = ws(ctx, name, (bytes), &q)) != GW_OK) return s;  \
        dst = (decltype(dst))q;                                   \
    } while (0)
    GW_WS("t_lev", sizeof(int32_t) * n_orb, d_lev);
    GW_WS("t_ph", sizeof(double) * n_orb, d_ph);
    GW_WS("t_start", sizeof(int32_t) * start.size(), d_start);
    GW_WS("t_pairs", sizeof(int32_t) * pbs.size(), d_pb);
    GW_WS("t_rho", sizeof(double) * std::max(Kp, Km) * nn, rho);
    GW_WS("t_F", sizeof(double) * 2 * Q * std::max(Kp, Km), F);
    GW_WS("t_G", sizeof(double) * nhb * 2 * Q, G);
    GW_WS("t_Rp", sizeof(double) * 2 * Q * nn, Rp);
    GW_WS("t_Rm", sizeof(double) * 2 * Q * nn, Rm);
    GW_WS("t_Ahat", sizeof(double) * 2 * (int64_t)qc * n_upper, Ahat);
    if (!a) GW_WS("t_a", sizeof(double) * nhb * n_upper, a);
    GW_WS("t_Kt", sizeof(zdbl) * 2 * g->n_omega, Kt);
    GW_WS("t_tw", sizeof(zdbl) * 2 * g->n_omega, tw);
#undef GW_WS
    GW_HIP(ctx, hipMemcpyAsync(d_lev, lev.data(), sizeof(int32_t) * n_orb, hipMemcpyHostToDevice, st));
    GW_HIP(ctx, hipMemcpyAsync(d_ph, ph.data(), sizeof(double) * n_orb, hipMemcpyHostToDevice, st));
    GW_HIP(ctx, hipMemcpyAsync(d_start, start.data(), sizeof(int32_t) * start.size(), hipMemcpyHostToDevice, st));
    GW_HIP(ctx, hipMemcpyAsync(d_pb, pbs.data(), sizeof(int32_t) * pbs.size(), hipMemcpyHostToDevice, st));
    GW_HIP(ctx, hipStreamSynchronize(st));  // the host vectors above are released on return
    // densities on the mesh and their transforms: Rp = F+ rho+, Rm = F- rhobar-
    GW_HIP(ctx, gwk::launch_rho_bins(st, n_orb, Kp, m->X, d_lev, d_ph, d_start, rho));
    GW_HIP(ctx, gwk::launch_dft_matrices(st, L, Q, Kp, F, 0, nullptr));
    GW_HIP(ctx, gwk::launch_dgemm(st, 2 * Q, (int)nn, Kp, 1.0, F, Kp, 0, rho, nn, 0, 0.0, Rp, nn, 0, 1));
    GW_HIP(ctx, gwk::launch_rho_bins(st, n_orb, Km, m->X, d_lev + nv, d_ph + nv, d_start + Kp + 1, rho));
    GW_HIP(ctx, gwk::launch_dft_matrices(st, L, Q, Km, F, nhb, G));
    GW_HIP(ctx, gwk::launch_dgemm(st, 2 * Q, (int)nn, Km, 1.0, F, Km, 0, rho, nn, 0, 0.0, Rm, nn, 0, 1));
    // time by time (in chunks): the local product, then its share of the
    // transform back, a = sum over chunks of G[:, chunk] Ahat[chunk]
    for (int q0 = 0; q0 < Q; q0 += qc) {
        const int nq = std::min(qc, Q - q0);
        GW_HIP(ctx, gwk::launch_time_contract(st, n_orb, n, class_off, q0, nq, m->blk_prod, m->blk_orb, m->orb_idx,
                                              m->blk_val, m->vals, d_pb, d_pb + npb, Rp, Rm, Ahat, cflops * nq));
        GW_HIP(ctx, gwk::launch_dgemm(st, nhb, (int)n_upper, 2 * nq, 1.0, G + 2 * q0, 2 * Q, 0, Ahat, n_upper, 0,
                                      q0 == 0 ? 0.0 : 1.0, a, n_upper, 0, 1));
    }
    const double dom = (g->omega_max - g->omega_min) / g->n_omega;
    GW_HIP(ctx, gwk::launch_kspec(st, g->n_omega, (int)std::lround(g->omega_min / dom), dom, g->eps, Kt, tw));
    if (v) {
        gwp::ARouteWs aw;
        if ((s = gwp::a_route_ws(ctx, "t_", n, nhb, g->n_omega, &aw)) != GW_OK) return s;
        s = gwp::a_from_bins_enqueue(ctx, st, n, g->n_omega, nhb, nullptr, nullptr, (const double *)a, v, aw, Kt, tw,
                                     (int)std::lround(g->omega_min / dom), dom, g->eps, chi0_out);
        if (s != GW_OK) return s;
    } else {
        GW_HIP(ctx, gwk::launch_fftconv(st, n, g->n_omega, nhb, (const double *)a, Kt, tw, (zdbl *)chi0_out));
    }
    if (rep) {
        GW_HIP(ctx, hipStreamSynchronize(st));
        std::memset(rep, 0, sizeof(*rep));
        rep->n_hbins = nhb;
        rep->frac_bits_used = 0;
        rep->n_dropped_pairs = dropped;
    }
    return GW_OK;
}

gw_status gw_build_chi0_time(gw_ctx *ctx, const gw_molecule *m, const gw_grid *g, void *stream, double *a_out,
                             void *chi0_out, gw_report *rep) {
    return build_time_impl(ctx, m, nullptr, g, stream, a_out, chi0_out, rep);
}

gw_status gw_build_A_time(gw_ctx *ctx, const gw_molecule *m, const double *v, const gw_grid *g, void *stream,
                          double *a_out, void *A_out, gw_report *rep) {
    if (ctx && !v) return fail(ctx, GW_E_INVALID, "v is NULL");
    return build_time_impl(ctx, m, v, g, stream, a_out, A_out, rep);
}

gw_status gw_self_energy(gw_ctx *ctx, const gw_molecule *m, const double *v, const gw_grid *g, const void *W,
                         void *stream, double *sigma_out, void *Sigma_out, double *Sigma_x_out, gw_report *rep) {
    if (!ctx) return GW_E_INVALID;
    if (ctx->sticky) return fail(ctx, GW_E_DEVICE, "context has a sticky device error: " + ctx->err);
    GW_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = as_stream(stream);
    if (!W || !Sigma_out) return fail(ctx, GW_E_INVALID, "W and Sigma_out must be set");
    if (Sigma_x_out && !v) return fail(ctx, GW_E_INVALID, "the exchange part needs v");
    int kbits = 0;
    gw_status s = check_grid(ctx, g, &kbits);
    if (s != GW_OK) return s;
    HostMol h;
    s = check_molecule(ctx, m, st, &h);
    if (s != GW_OK) return s;
    const int n_orb = m->n_orb, n_occ = m->n_occ, n = m->n_prod, nblk = m->n_blk;
    if (h.max_o > TIME_MAX_ORB)
        return fail(ctx, GW_E_INVALID, "the self-energy takes orbital sets of at most " +
                                           std::to_string(TIME_MAX_ORB) + " orbitals");
    const int N = g->n_omega, n_sb = N / 2;
    const double d = (g->omega_max - g->omega_min) / N;
    LevelTables lt;
    s = level_tables(ctx, h, n_orb, n_occ, kbits, n_sb, &lt);
    if (s != GW_OK) return s;
    const int nv = lt.nv, Kp = lt.Kp, Km = lt.Km;
    // the convolutions of rho+- (Kp, Km bins) with gamma (n_sb bins): the
    // cyclic transform of length L has no wrap-around
    const int L = std::max(Kp, Km) + n_sb - 1;
    const int Q = L / 2 + 1;
    std::vector<int32_t> pbs;
    int max_vblock = 0, class_off[5];
    const int npb = block_pairs(h, nblk, &pbs, &max_vblock, class_off);
    double cflops = 0.0;
    for (int b1 = 0; b1 < nblk; ++b1)
        for (int b2 = b1; b2 < nblk; ++b2) {
            const double n1 = h.blk_orb[b1 + 1] - h.blk_orb[b1], n2 = h.blk_orb[b2 + 1] - h.blk_orb[b2];
            const double pm = h.blk_prod[b1 + 1] - h.blk_prod[b1], pn = h.blk_prod[b2 + 1] - h.blk_prod[b2];
            cflops += pm * (4.0 * pn * n2 * n2 + 16.0 * n1 * n2 * n2 + 8.0 * n1 * n1 * n2);
        }
    const int64_t nn = (int64_t)n_orb * n_orb;
    const int64_t n_upper = (int64_t)n * (n + 1) / 2;
    // time points per chunk: transformed gamma and the two products within 4 GiB
    const int qc = (int)std::max<int64_t>(1, std::min<int64_t>(Q, (int64_t)(4ll << 30) / (16 * n_upper + 32 * nn)));
    void *q;
    int32_t *d_lev, *d_start, *d_pb;
    double *d_ph, *rho, *F, *Gi, *Rp, *Rm, *gam, *Gh, *S, *sig = sigma_out, *Xt = nullptr;
    zdbl *Kpm;
    const int kf = std::max(std::max(Kp, Km), n_sb);
#define GW_WS(name, bytes, dst)                                   \
    do {                                                          \
        if ((s = ws(ctx, name, (bytes), &q)) != GW_OK) return s;  \
        dst = (decltype(dst))q;                                   \
    } while (0)
    GW_WS("s_lev", sizeof(int32_t) * n_orb, d_lev);
    GW_WS("s_ph", sizeof(double) * n_orb, d_ph);
    GW_WS("s_start", sizeof(int32_t) * lt.start.size(), d_start);
    GW_WS("s_pairs", sizeof(int32_t) * pbs.size(), d_pb);
    GW_WS("s_rho", sizeof(double) * std::max(std::max(Kp, Km), 1) * nn, rho);
    GW_WS("s_F", sizeof(double) * 2 * Q * kf, F);
    GW_WS("s_Ginv", sizeof(double) * n_sb * 2 * Q, Gi);
    GW_WS("s_Rp", sizeof(double) * 2 * Q * nn, Rp);
    GW_WS("s_Rm", sizeof(double) * 2 * Q * nn, Rm);
    GW_WS("s_gam", sizeof(double) * n_sb * n_upper, gam);
    GW_WS("s_Gh", sizeof(double) * 2 * (int64_t)qc * n_upper, Gh);
    GW_WS("s_S", sizeof(double) * 4 * (int64_t)qc * nn, S);
    if (!sig) GW_WS("s_sigma", sizeof(double) * 2 * n_sb * nn, sig);
    GW_WS("s_Kpm", sizeof(zdbl) * 2 * (int64_t)N * n_sb, Kpm);
    if (Sigma_x_out) GW_WS("s_Xt", sizeof(double) * nn, Xt);
#undef GW_WS
    GW_HIP(ctx, hipMemcpyAsync(d_lev, lt.lev.data(), sizeof(int32_t) * n_orb, hipMemcpyHostToDevice, st));
    GW_HIP(ctx, hipMemcpyAsync(d_ph, lt.ph.data(), sizeof(double) * n_orb, hipMemcpyHostToDevice, st));
    GW_HIP(ctx, hipMemcpyAsync(d_start, lt.start.data(), sizeof(int32_t) * lt.start.size(), hipMemcpyHostToDevice,
                               st));
    GW_HIP(ctx, hipMemcpyAsync(d_pb, pbs.data(), sizeof(int32_t) * pbs.size(), hipMemcpyHostToDevice, st));
    GW_HIP(ctx, hipStreamSynchronize(st));  // the host tables above are released on return
    double *Sp = S, *Sm = S + 2 * (int64_t)qc * nn;
    double *sig_p = sig, *sig_m = sig + (int64_t)n_sb * nn;
    // the densities and gamma in time
    GW_HIP(ctx, gwk::launch_rho_bins(st, n_orb, Kp, m->X, d_lev, d_ph, d_start, rho));
    GW_HIP(ctx, gwk::launch_dft_matrices(st, L, Q, Kp, F, 0, nullptr));
    GW_HIP(ctx, gwk::launch_dgemm(st, 2 * Q, (int)nn, Kp, 1.0, F, Kp, 0, rho, nn, 0, 0.0, Rp, nn, 0, 1));
    GW_HIP(ctx, gwk::launch_rho_bins(st, n_orb, Km, m->X, d_lev + nv, d_ph + nv, d_start + Kp + 1, rho));
    GW_HIP(ctx, gwk::launch_dft_matrices(st, L, Q, Km, F, n_sb, Gi));
    GW_HIP(ctx, gwk::launch_dgemm(st, 2 * Q, (int)nn, Km, 1.0, F, Km, 0, rho, nn, 0, 0.0, Rm, nn, 0, 1));
    GW_HIP(ctx, gwk::launch_w_spectral(st, n, n_sb, (int)std::lround(-g->omega_min / d), d, (const zdbl *)W, gam));
    GW_HIP(ctx, gwk::launch_dft_matrices(st, L, Q, n_sb, F, 0, nullptr));
    for (int q0 = 0; q0 < Q; q0 += qc) {
        const int nq = std::min(qc, Q - q0);
        GW_HIP(ctx, gwk::launch_dgemm(st, 2 * nq, (int)n_upper, n_sb, 1.0, F + (int64_t)2 * q0 * n_sb, n_sb, 0, gam,
                                      n_upper, 0, 0.0, Gh, n_upper, 0, 1));
        GW_HIP(ctx, gwk::launch_fill_u64(st, (uint64_t *)S, 4 * (int64_t)nq * nn, 0));
        Sm = S + 2 * (int64_t)nq * nn;
        GW_HIP(ctx, gwk::launch_sigma_contract(st, n_orb, n, class_off, q0, nq, m->blk_prod, m->blk_orb, m->orb_idx,
                                               m->blk_val, m->vals, d_pb, d_pb + npb, Rp, Rm, Gh, Sp, Sm,
                                               max_vblock, cflops * nq));
        const double beta = q0 == 0 ? 0.0 : 1.0;
        GW_HIP(ctx, gwk::launch_dgemm(st, n_sb, (int)nn, 2 * nq, 1.0, Gi + 2 * q0, 2 * Q, 0, Sp, nn, 0, beta, sig_p,
                                      nn, 0, 1));
        GW_HIP(ctx, gwk::launch_dgemm(st, n_sb, (int)nn, 2 * nq, 1.0, Gi + 2 * q0, 2 * Q, 0, Sm, nn, 0, beta, sig_m,
                                      nn, 0, 1));
    }
    // Sigma(omega_j + i eps) = Kp sigma+ + Km sigma-
    zdbl *Kp_ = Kpm, *Km_ = Kpm + (int64_t)N * n_sb;
    GW_HIP(ctx, gwk::launch_cauchy_pm(st, N, n_sb, g->omega_min, d, g->eps, Kp_, Km_));
    GW_HIP(ctx, gwk::launch_zdgemm(st, N, (int)nn, n_sb, 1.0, Kp_, n_sb, 0, sig_p, nn, 0, 0.0, (zdbl *)Sigma_out, nn,
                                   0, 1));
    GW_HIP(ctx, gwk::launch_zdgemm(st, N, (int)nn, n_sb, 1.0, Km_, n_sb, 0, sig_m, nn, 0, 1.0, (zdbl *)Sigma_out, nn,
                                   0, 1));
    if (Sigma_x_out) {
        // exchange: the same contraction once, with the occupied density
        // matrix D = X_occ X_occ^T for rho and v for gamma (both real)
        GW_HIP(ctx, gwk::launch_transpose_d(st, n_orb, n_orb, m->X, Xt));
        GW_HIP(ctx, gwk::launch_fill_u64(st, (uint64_t *)Rp, 2 * nn, 0));
        GW_HIP(ctx, gwk::launch_dgemm(st, n_orb, n_orb, n_occ, 1.0, m->X, n_orb, 0, Xt, n_orb, 0, 0.0, Rp, n_orb, 0,
                                      1));
        GW_HIP(ctx, gwk::launch_fill_u64(st, (uint64_t *)Gh, 2 * n_upper, 0));
        GW_HIP(ctx, gwk::launch_pack_upper(st, n, v, Gh));
        GW_HIP(ctx, gwk::launch_fill_u64(st, (uint64_t *)S, 2 * nn, 0));
        GW_HIP(ctx, gwk::launch_sigma_contract(st, n_orb, n, class_off, 0, 1, m->blk_prod, m->blk_orb, m->orb_idx,
                                               m->blk_val, m->vals, d_pb, d_pb + npb, Rp, nullptr, Gh, S, nullptr,
                                               max_vblock, cflops / 4));
        GW_HIP(ctx, gwk::launch_scale_copy(st, nn, -1.0, S, Sigma_x_out));
    }
    if (rep) {
        GW_HIP(ctx, hipStreamSynchronize(st));
        std::memset(rep, 0, sizeof(*rep));
        rep->n_hbins = n_sb;
    }
    return GW_OK;
}

gw_status gw_dyson_dos(gw_ctx *ctx, const gw_molecule *m, const gw_grid *g, const void *Sigma_c,
                       const double *Sigma_x, const double *Vxc, void *stream, double *dos_out, void *G_out,
                       gw_report *rep) {
    if (!ctx) return GW_E_INVALID;
    if (ctx->sticky) return fail(ctx, GW_E_DEVICE, "context has a sticky device error: " + ctx->err);
    GW_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = as_stream(stream);
    if (!dos_out) return fail(ctx, GW_E_INVALID, "dos_out is NULL");
    int kbits = 0;
    gw_status s = check_grid(ctx, g, &kbits);
    if (s != GW_OK) return s;
    HostMol h;
    s = check_molecule(ctx, m, st, &h);
    if (s != GW_OK) return s;
    const int n = m->n_orb, N = g->n_omega;
    const int64_t nn = (int64_t)n * n;
    const double d = (g->omega_max - g->omega_min) / N;
    void *q;
    double *Xe, *Xt, *H, *Hs, *ones;
#define GW_WS(name, bytes, dst)                                   \
    do {                                                          \
        if ((s = ws(ctx, name, (bytes), &q)) != GW_OK) return s;  \
        dst = (decltype(dst))q;                                   \
    } while (0)
    GW_WS("d_Xe", sizeof(double) * nn, Xe);
    GW_WS("d_Xt", sizeof(double) * nn, Xt);
    GW_WS("d_H", sizeof(double) * nn, H);
    GW_WS("d_Hs", sizeof(double) * nn, Hs);
    GW_WS("d_ones", sizeof(double) * n, ones);
    gwp::SolvePlan p;
    s = gwp::solve_plan(ctx, n, N, false, "d_", &p);
    if (s != GW_OK) return s;
    zdbl *Gws = nullptr;
    if (!G_out) GW_WS("d_G", sizeof(zdbl) * (size_t)p.nbmax * nn, Gws);
#undef GW_WS
    // H_KS = X diag(E) X^T (orthonormal orbitals), then the static part
    // H_KS + Sigma_x - V_xc
    GW_HIP(ctx, gwk::launch_scale_cols(st, n, m->X, m->eig, Xe));
    GW_HIP(ctx, gwk::launch_transpose_d(st, n, n, m->X, Xt));
    GW_HIP(ctx, gwk::launch_dgemm(st, n, n, n, 1.0, Xe, n, 0, Xt, n, 0, 0.0, H, n, 0, 1));
    GW_HIP(ctx, gwk::launch_static_part(st, nn, H, Sigma_x, Vxc, Hs));
    GW_HIP(ctx, gwk::launch_fill_u64(st, (uint64_t *)ones, n, 0x3FF0000000000000ull));  // 1.0
    gwp::SolveWs &w = p.w;
    for (int j0 = 0; j0 < N; j0 += p.nbmax) {
        const int nb = std::min(p.nbmax, N - j0);
        zdbl *G = G_out ? (zdbl *)G_out + (int64_t)j0 * nn : Gws;
        GW_HIP(ctx, gwk::launch_dyson_form(st, n, j0, nb, g->omega_min, d, g->eps, Hs, (const zdbl *)Sigma_c, w.A));
        GW_HIP(ctx, gwk::launch_fill_u32(st, (uint32_t *)w.info, nb, 0u));
        GW_HIP(ctx, gwk::getrf_batched<zdbl>(st, n, w.A, nn, w.ipiv, (zdbl *)w.Li, (zdbl *)w.Ui, (zdbl *)w.scratch,
                                             w.info, nb));
        GW_HIP(ctx, gwk::launch_perm(st, n, w.ipiv, w.perm, nb));
        GW_HIP(ctx, gwk::launch_init_rhs_perm(st, n, ones, 1, w.perm, G, nn, nb));  // P 1
        GW_HIP(ctx, gwk::getrs_batched<zdbl>(st, n, n, w.A, nn, w.ipiv, (const zdbl *)w.Li, (const zdbl *)w.Ui, G,
                                             nn, nb, false));
        GW_HIP(ctx, gwk::launch_trace_dos(st, n, j0, nb, G, nn, dos_out));
    }
    if (rep) {
        GW_HIP(ctx, hipStreamSynchronize(st));
        std::memset(rep, 0, sizeof(*rep));
        rep->n_solved = N;
    }
    return GW_OK;
}

}  // extern "C"

namespace {
// W from chi0 (X0) or from A = 1 - v chi0 (Ain); exactly one is given.
gw_status solve_W_impl(gw_ctx *ctx, const double *v, int32_t v_is_diag, int32_t n, const zdbl *X0, zdbl *Ain,
                       int32_t n_omega, gw_precision prec, double tol, void *stream, void *W_out, gw_report *rep) {
    if (!ctx) return GW_E_INVALID;
    if (ctx->sticky) return fail(ctx, GW_E_DEVICE, "context has a sticky device error: " + ctx->err);
    GW_HIP(ctx, hipSetDevice(ctx->device));
    if (!v || (!X0 && !Ain) || !W_out) return fail(ctx, GW_E_INVALID, "NULL pointer argument");
    if (n < 1 || n > 32768) return fail(ctx, GW_E_INVALID, "n must be in [1, 32768]");
    if (n_omega < 2 || (n_omega & 1)) return fail(ctx, GW_E_INVALID, "n_omega must be even and >= 2");
    if (prec != GW_FP64 && prec != GW_FP32_IR && prec != GW_BF16X_IR)
        return fail(ctx, GW_E_INVALID, "unknown precision");
    if (prec != GW_FP64 && !(tol > 0.0)) return fail(ctx, GW_E_INVALID, "tol must be positive for mixed precision");
    hipStream_t st = as_stream(stream);
    const bool mixed = prec != GW_FP64;
    const int64_t nn = (int64_t)n * n;
    gwp::Bf16xScope bf16x(prec == GW_BF16X_IR);
    gwp::SolvePlan p;
    gw_status s = gwp::solve_plan(ctx, n, n_omega, mixed, "", &p);
    if (s != GW_OK) return s;
    zdbl *W = (zdbl *)W_out;
    int n_solved = 0, n_fallback = 0, max_it = 0;
    double max_rel = 0.0;
    if (!mixed) {
        // one stream by default: every kernel then has the whole machine (the
        // panel kernel needs a whole CU, which a second stream's GEMM
        // workgroups keep occupied); GW_SOLVE_STREAMS=2 overlaps one frequency
        // batch's panels with the other batch's products
        int nstreams = 1;
        if (const char *e = std::getenv("GW_SOLVE_STREAMS")) nstreams = std::max(1, std::min(2, std::atoi(e)));
        if (ctx->own_stream || n_omega < 8) nstreams = 1;
        if (nstreams == 1) {
            // the lone point j = 0 (no mirror partner) is a batch of one: its
            // panels would hold one CU each while the rest of the chip idles,
            // so it runs on the context's second stream beside the batches
            bool side = !ctx->own_stream && n_omega >= 8;
            gwp::SolvePlan p0;
            if (side && (s = gwp::solve_plan(ctx, n, 2, false, "j0", &p0)) != GW_OK) {
                if (s != GW_E_OOM) return s;
                side = false;  // no room for a second workspace: j = 0 stays in order
            }
            if (side) {
                if ((s = aux_stream(ctx)) != GW_OK) return s;
                GW_HIP(ctx, hipEventRecord(ctx->fork_ev, st));
                GW_HIP(ctx, hipStreamWaitEvent(ctx->aux, ctx->fork_ev, 0));
                gwp::SolveWs w0;
                if ((s = gwp::batch_ws(ctx, ctx->aux, p0.w, Ain, W, nn, 0, 1, &w0)) != GW_OK) return s;
                if ((s = gwp::solve_batch_fp64(ctx, ctx->aux, n, v, v_is_diag, X0, W, 1, w0)) != GW_OK) return s;
                GW_HIP(ctx, hipEventRecord(ctx->join_ev, ctx->aux));
            }
            s = gwp::solve_enqueue_nosync(ctx, p, st, v, v_is_diag, X0, W, 0, Ain, side);
            if (s != GW_OK) return s;
            if (side) GW_HIP(ctx, hipStreamWaitEvent(st, ctx->join_ev, 0));
            for (auto &bt : freq_batches(n_omega, p.nbmax)) n_solved += bt.second;
        } else {
            // frequency batches alternate between the caller's stream and a
            // second one, so that one batch's latency-bound panels overlap the
            // other's matrix-core products; each stream has its own workspace
            gwp::SolvePlan p2[2];
            if ((s = gwp::solve_plan(ctx, n, n_omega, false, "", &p2[0], ctx->budget / 2)) != GW_OK) return s;
            if ((s = gwp::solve_plan(ctx, n, n_omega, false, "t1", &p2[1], ctx->budget / 2)) != GW_OK) return s;
            if ((s = aux_stream(ctx)) != GW_OK) return s;
            hipStream_t ss[2] = {ctx->aux, st};
            GW_HIP(ctx, hipEventRecord(ctx->fork_ev, st));
            GW_HIP(ctx, hipStreamWaitEvent(ctx->aux, ctx->fork_ev, 0));
            const auto bts = freq_batches(n_omega, std::max(1, std::min(p2[0].nbmax, (n_omega / 2 + 1) / 2)));
            for (size_t i = 0; i < bts.size(); ++i) {
                const int j0 = bts[i].first, nb = bts[i].second, q = (int)(i % 2);
                gwp::SolveWs wb;
                if ((s = gwp::batch_ws(ctx, ss[q], p2[q].w, Ain, W, nn, j0, nb, &wb)) != GW_OK) return s;
                s = gwp::solve_batch_fp64(ctx, ss[q], n, v, v_is_diag, X0 ? X0 + j0 * nn : nullptr, W + j0 * nn, nb,
                                          wb);
                if (s != GW_OK) return s;
                n_solved += nb;
            }
            GW_HIP(ctx, hipEventRecord(ctx->join_ev, ctx->aux));
            GW_HIP(ctx, hipStreamWaitEvent(st, ctx->join_ev, 0));
            if (n_omega >= 4) GW_HIP(ctx, gwk::launch_conj_mirror(st, nn, n_omega, W));
        }
    } else {
        for (auto &bt : freq_batches(n_omega, p.nbmax)) {
            const int j0 = bt.first, nb = bt.second;
            n_solved += nb;
            std::vector<int> its;
            std::vector<double> rel;
            gwp::SolveWs wb;
            if ((s = gwp::batch_ws(ctx, st, p.w, Ain, W, nn, j0, nb, &wb)) != GW_OK) return s;
            s = solve_batch_mixed(ctx, st, n, v, v_is_diag, X0 ? X0 + j0 * nn : nullptr, W + j0 * nn, nb, tol, wb,
                                  &its, &rel, 6);
            if (s != GW_OK) return s;
            for (int b = 0; b < nb; ++b) {
                if (its[b] < 0) {
                    // not converged: FP64 fallback for this frequency, from the FP64
                    // A of the batch (chi0 may already be overwritten in place)
                    ++n_fallback;
                    gwp::SolvePlan p64;
                    if ((s = gwp::solve_plan(ctx, n, 2, false, "fb", &p64)) != GW_OK) return s;
                    GW_HIP(ctx, hipMemcpyAsync(p64.w.A, wb.A + (int64_t)b * nn, (size_t)nn * 16,
                                               hipMemcpyDeviceToDevice, st));
                    s = gwp::solve_batch_fp64(ctx, st, n, v, v_is_diag, nullptr, W + (j0 + b) * nn, 1, p64.w);
                    if (s != GW_OK) return s;
                } else {
                    max_it = std::max(max_it, its[b]);
                    max_rel = std::max(max_rel, rel[b]);
                }
            }
        }
        if (n_omega >= 4) GW_HIP(ctx, gwk::launch_conj_mirror(st, nn, n_omega, W));
    }
    if (rep) {
        GW_HIP(ctx, hipStreamSynchronize(st));
        rep->n_solved = n_solved;
        rep->n_fallback = n_fallback;
        rep->max_iter = max_it;
        rep->max_rel_update = max_rel;
    }
    return GW_OK;
}
}  // namespace

extern "C" {
gw_status gw_solve_W(gw_ctx *ctx, const double *v, int32_t v_is_diag, int32_t n, const void *chi0, int32_t n_omega,
                     gw_precision prec, double tol, void *stream, void *W_out, gw_report *rep) {
    if (ctx && !chi0) return fail(ctx, GW_E_INVALID, "NULL pointer argument");
    return solve_W_impl(ctx, v, v_is_diag, n, (const zdbl *)chi0, nullptr, n_omega, prec, tol, stream, W_out, rep);
}

gw_status gw_solve_W_A(gw_ctx *ctx, const double *v, int32_t v_is_diag, int32_t n, void *A, int32_t n_omega,
                       gw_precision prec, double tol, void *stream, void *W_out, gw_report *rep) {
    if (ctx && !A) return fail(ctx, GW_E_INVALID, "NULL pointer argument");
    return solve_W_impl(ctx, v, v_is_diag, n, nullptr, (zdbl *)A, n_omega, prec, tol, stream, W_out, rep);
}

// The A route for gw_build_A (basis = NULL) and gw_build_A_compressed.
static gw_status build_A_impl(gw_ctx *ctx, const gw_molecule *m, const double *v, const gw_grid *g, const double *basis,
                       int32_t k, void *stream, void *A_out, gw_report *rep) {
    if (!ctx) return GW_E_INVALID;
    if (ctx->sticky) return fail(ctx, GW_E_DEVICE, "context has a sticky device error: " + ctx->err);
    GW_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = as_stream(stream);
    if (!v || !A_out || !g) return fail(ctx, GW_E_INVALID, "NULL pointer argument");
    if (!gwp::a_mesh_ok(g->n_omega))
        return fail(ctx, GW_E_INVALID, "the A route with GW_A_TRANSFORM=fft needs n_omega in [128, 1024]");
    gwp::BuildPlan p;
    gw_status s = gwp::build_plan(ctx, m, g, basis, k, st, "", nullptr, &p);
    if (s != GW_OK) return s;
    gwp::ARouteWs aw;
    if ((s = gwp::a_route_ws(ctx, "", p.rows, p.nhb, g->n_omega, &aw)) != GW_OK) return s;
    const bool kspec = ctx->ks_n != g->n_omega || ctx->ks_min != g->omega_min || ctx->ks_d != p.dom ||
                       ctx->ks_eps != g->eps;
    if ((s = gwp::a_route_enqueue(ctx, p, st, v, aw, kspec, A_out)) != GW_OK) return s;
    if (kspec) {
        ctx->ks_n = g->n_omega;
        ctx->ks_min = g->omega_min;
        ctx->ks_d = p.dom;
        ctx->ks_eps = g->eps;
    }
    if (rep) {
        int64_t hs[2];
        int32_t sv = 0;
        GW_HIP(ctx, hipMemcpyAsync(hs, p.stat, sizeof(hs), hipMemcpyDeviceToHost, st));
        GW_HIP(ctx, hipMemcpyAsync(&sv, p.sdev, sizeof(sv), hipMemcpyDeviceToHost, st));
        GW_HIP(ctx, hipStreamSynchronize(st));
        std::memset(rep, 0, sizeof(*rep));
        rep->n_hbins = p.nhb;
        rep->frac_bits_used = sv;
        rep->n_dropped_pairs = hs[1];
    }
    return GW_OK;
}

gw_status gw_build_A(gw_ctx *ctx, const gw_molecule *m, const double *v, const gw_grid *g, void *stream,
                     void *A_out, gw_report *rep) {
    return build_A_impl(ctx, m, v, g, nullptr, 0, stream, A_out, rep);
}

gw_status gw_build_A_compressed(gw_ctx *ctx, const gw_molecule *m, const double *S, const double *basis, int32_t k,
                                const gw_grid *g, void *stream, void *A_out, gw_report *rep) {
    if (ctx && (!basis || k < 1)) return fail(ctx, GW_E_INVALID, "gw_build_A_compressed needs a basis and k >= 1");
    return build_A_impl(ctx, m, S, g, basis, k, stream, A_out, rep);
}


gw_status gw_compress_basis(gw_ctx *ctx, const double *v, int32_t n, int32_t k, void *stream, double *Q_out,
                            double *S_out) {
    if (!ctx) return GW_E_INVALID;
    if (ctx->sticky) return fail(ctx, GW_E_DEVICE, "context has a sticky device error: " + ctx->err);
    if (!v || !Q_out || !S_out || n < 1 || k < 1 || k > n) return fail(ctx, GW_E_INVALID, "bad compress arguments");
    GW_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = as_stream(stream);
    void *work;
    gw_status s;
    if ((s = ws(ctx, "cWork", sizeof(double) * gwk::compress_work_doubles(n, k), &work)) != GW_OK) return s;
    hipError_t e = gwk::compress_basis(st, n, k, v, Q_out, S_out, (double *)work, 4);
    if (e == hipErrorUnknown) return fail(ctx, GW_E_NOCONV, "subspace iteration lost a direction (v not finite?)");
    GW_HIP(ctx, e);
    return GW_OK;
}

gw_status gw_pair_basis(gw_ctx *ctx, const gw_molecule *m, const double *v, double e_threshold, int32_t k,
                        void *stream, double *Z_out, double *U_out, double *R_out, int64_t *n_rank_out) {
    if (!ctx) return GW_E_INVALID;
    if (ctx->sticky) return fail(ctx, GW_E_DEVICE, "context has a sticky device error: " + ctx->err);
    if (!v || !Z_out || !U_out || k < 1) return fail(ctx, GW_E_INVALID, "bad pair-basis arguments");
    if (!(e_threshold > 0.0) || !std::isfinite(e_threshold))
        return fail(ctx, GW_E_INVALID, "e_threshold must be positive and finite");
    GW_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = as_stream(stream);
    HostMol h;
    gw_status s = check_molecule(ctx, m, st, &h);
    if (s != GW_OK) return s;
    const int n = m->n_prod, n_occ = m->n_occ, n_virt = m->n_orb - m->n_occ;
    if (k > n) return fail(ctx, GW_E_INVALID, "k must not exceed n_prod");
    // pairs with F - E < e_threshold: for each occupied E a prefix of the
    // empty states (eigenvalues ascend), and the prefix grows with E
    std::vector<int32_t> src;
    std::vector<int64_t> off(n_occ + 1, 0);
    for (int e = 0; e < n_occ; ++e) {
        int c = 0;
        while (c < n_virt && h.eig[n_occ + c] - h.eig[e] < e_threshold) ++c;
        off[e + 1] = off[e] + c;
        for (int f = 0; f < c; ++f) src.push_back((int32_t)((int64_t)e * n_virt + f));
    }
    const int64_t nr = off[n_occ];
    if (n_rank_out) *n_rank_out = nr;
    if (nr < k) return fail(ctx, GW_E_INVALID, "fewer pairs below the threshold (" + std::to_string(nr) + ") than k");
    if (nr > 65536) return fail(ctx, GW_E_INVALID, "more than 65536 pairs below the threshold");
    // pair vectors of the occupied states that have selected pairs, in chunks
    int e_first = 0;
    while (off[e_first + 1] == 0) ++e_first;
    const int64_t cap = std::max<int64_t>(1, ((int64_t)1 << 31) / (8 * (int64_t)n * n_virt));
    const int echunk = (int)std::min<int64_t>(n_occ - e_first, cap);
    void *Pc, *Xg, *srcd, *work;
    if ((s = ws(ctx, "pbP", sizeof(double) * (size_t)n * echunk * n_virt, &Pc)) != GW_OK) return s;
    if ((s = ws(ctx, "pbX", sizeof(double) * (size_t)n * nr, &Xg)) != GW_OK) return s;
    if ((s = ws(ctx, "pbSrc", sizeof(int32_t) * (size_t)nr, &srcd)) != GW_OK) return s;
    if ((s = ws(ctx, "pbWork", sizeof(double) * gwk::pair_basis_work_doubles(n, (int)nr, k), &work)) != GW_OK)
        return s;
    GW_HIP(ctx, hipMemcpyAsync(srcd, src.data(), sizeof(int32_t) * nr, hipMemcpyHostToDevice, st));
    for (int e0 = e_first; e0 < n_occ; e0 += echunk) {
        const int ec = std::min(echunk, n_occ - e0);
        const int64_t cw = (int64_t)ec * n_virt;
        GW_HIP(ctx, gwk::launch_pairvec(st, m->n_orb, n_occ, n, m->n_blk, m->X, m->blk_prod, m->blk_orb, m->orb_idx,
                                        m->blk_val, m->vals, h.max_o, e0, ec, cw, (double *)Pc));
        GW_HIP(ctx, gwk::launch_gather_cols(st, n, (int)(off[e0 + ec] - off[e0]), cw, (const double *)Pc,
                                            (const int32_t *)srcd, (int64_t)e0 * n_virt, (int)off[e0],
                                            (double *)Xg, nr));
    }
    hipError_t e = gwk::pair_basis(st, n, (int)nr, k, v, (const double *)Xg, Z_out, U_out, R_out, (double *)work, 4);
    if (e == hipErrorUnknown)
        return fail(ctx, GW_E_NOCONV, "k exceeds the rank of the generating pair vectors (or v is not finite)");
    GW_HIP(ctx, e);
    return GW_OK;
}

gw_status gw_decompress(gw_ctx *ctx, const double *U, int32_t n, int32_t k, const void *X, const double *R,
                        void *stream, void *W_out) {
    if (!ctx) return GW_E_INVALID;
    if (ctx->sticky) return fail(ctx, GW_E_DEVICE, "context has a sticky device error: " + ctx->err);
    if (!U || !X || !W_out || n < 1 || k < 1 || k > n) return fail(ctx, GW_E_INVALID, "bad decompress arguments");
    GW_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = as_stream(stream);
    void *T, *Ut;
    gw_status s;
    if ((s = ws(ctx, "dT", sizeof(zdbl) * (int64_t)n * k, &T)) != GW_OK) return s;
    if ((s = ws(ctx, "dUt", sizeof(double) * (int64_t)n * k, &Ut)) != GW_OK) return s;
    GW_HIP(ctx, gwk::launch_transpose_d(st, n, k, U, (double *)Ut));
    // T = U X ([n][k]), W = T U^T ([n][n]) (Section 8.B decompression)
    GW_HIP(ctx, gwk::launch_dzgemm(st, n, k, k, 1.0, U, k, 0, (const zdbl *)X, k, 0, 0.0, (zdbl *)T, k, 0, 1));
    if (R) GW_HIP(ctx, gwk::launch_init_rhs(st, n, R, 0, (zdbl *)W_out, 0, 1));
    GW_HIP(ctx, gwk::launch_zdgemm(st, n, n, k, 1.0, (const zdbl *)T, k, 0, (const double *)Ut, n, 0, R ? 1.0 : 0.0,
                                   (zdbl *)W_out, n, 0, 1));
    return GW_OK;
}

}  // extern "C"

// Free every workspace buffer of a context (serving slots do this after each
// request so that admission can count transient memory exactly).
void gwk_ctx_trim(gw_ctx *c) {
    if (c->own_stream) {
        for (auto &kv : c->bufs)
            if (kv.second.ptr) (void)hipFreeAsync(kv.second.ptr, c->own_stream);
    } else {
        (void)hipDeviceSynchronize();
        for (auto &kv : c->bufs)
            if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    }
    c->bufs.clear();
    c->ks_n = 0;
}

// Stream-ordered allocation from the device's pool.  The pool keeps freed
// memory for reuse; when it cannot satisfy a request from that cache (sizes
// differ) and the device is out of memory, the cache is handed back to the
// device and the allocation tried once more.
hipError_t gwk_malloc_async(void **p, size_t bytes, hipStream_t st) {
    if (gwp::fault() == gwp::FAULT_OOM) return hipErrorOutOfMemory;
    hipError_t e = hipMallocAsync(p, bytes, st);
    if (e != hipErrorOutOfMemory) return e;
    (void)hipGetLastError();
    int dev = 0;
    hipMemPool_t pool = nullptr;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetDefaultMemPool(&pool, dev) != hipSuccess || !pool) return e;
    (void)hipStreamSynchronize(st);
    (void)hipMemPoolTrimTo(pool, 0);
    return hipMallocAsync(p, bytes, st);
}

size_t gwk_ctx_bytes(const gw_ctx *c) {
    size_t b = 0;
    for (auto &kv : c->bufs) b += kv.second.bytes;
    return b;
}

size_t gwk_solve_ws_bytes(int n, int n_omega, bool mixed, size_t budget) { return solve_ws_bytes(n, n_omega, mixed, budget); }
