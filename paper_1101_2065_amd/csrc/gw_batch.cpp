// Batched form: many molecules of different sizes on one mesh, recorded once
// into a hipGraph and replayed.
//
// gw_batch_create validates and plans every molecule (the only host
// synchronisation), sizes the shared workspaces (two planning passes, so
// every recorded pointer is final), picks GEMM tile shapes per size class
// from the autotuner table, then records: all chi0 builds on the caller's
// stream, then the molecules' W solves spread over parallel stream branches
// (fork/join through events), so solves of different molecules run
// concurrently.  gw_batch_run replays the graph; for the mixed form it then
// checks every frequency's last refinement steps and re-solves in FP64 (outside
// the graph) any frequency that did not reach the tolerance.
#include "gw_plan.h"
#include "gw_tune.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace gwk {
hipError_t launch_fill_u32(hipStream_t st, uint32_t *p, int64_t n, uint32_t value);
}

using gwp::fail;

struct gw_batch {
    gw_ctx *ctx = nullptr;
    int n_mol = 0;
    std::vector<gw_molecule> mols;
    std::vector<const double *> v;
    std::vector<void *> chi0, W;
    std::vector<int> n, tile;
    gw_grid g{};
    gw_precision prec = GW_FP64;
    double tol = 1e-7;
    int n_refine = 0;
    std::vector<double *> norms;  // per molecule [2][n_omega][2] (last two refinement steps)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;  // private stream the graph is recorded on
    std::vector<hipStream_t> branches;
    std::vector<hipEvent_t> events;
    uint64_t generation = 0;  // the context's batch generation this graph was recorded in
    int mode = 1;             // 0: molecules on parallel branches; 1, 2: lock steps (1: aligned at the end)
    gwp::LockStepStats ls_stats;
};

namespace {

// ------------------------------------------------------------------ autotuner
// Table: (precision, size class) -> tile of the long complex products of the
// LU and the solves (0: 64x64 K16, 1: 128x64 K8, 2: 64x32 K8, 3: 128x32 K8).
// The size class is n rounded up to a multiple of 256; the precision is that
// of the factorisation (FP64, or FP32 for both mixed forms: under BF16x the
// rank-K trailing updates run on the split-BF16 kernel, and the FP32 table
// entry serves its remaining complex-float products).  A class is measured the
// first time it is seen, on the molecule's own first trailing update
// (M = N = n - 256, K = 256, a batch of up to four frequencies): one warm-up
// launch and five timed ones per tile, the median kept.  The table lives in
// memory and in a JSON file ($GW_TUNE_FILE, default $HOME/.cache/gw_tune.json).
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

std::string tune_key(int cls, gw_precision prec) {
    return std::string(prec == GW_FP64 ? "zgemm_fp64" : "cgemm_fp32") + "_n" + std::to_string(cls);
}

gw_status tune_tile(gw_ctx *ctx, int n, gw_precision prec, hipStream_t st, int *tile) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const std::string path = gwt::cache_path();
    if (!g_tune_loaded) {
        g_tune_loaded = true;
        std::string err;
        if (!gwt::load(path, &g_tune, &err)) ctx->err = "autotuner table not read (" + err + "); measuring afresh";
    }
    const int cls = ((n + 255) / 256) * 256;
    const std::string key = tune_key(cls, prec);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
        *tile = it->second;
        return GW_OK;
    }
    if (n <= 256) {  // no long products at this size
        *tile = 3;
        g_tune[key] = 3;
        return GW_OK;
    }
    const bool dbl = prec == GW_FP64;
    const int M = n - 256, K = 256, batch = 4;
    const size_t esz = dbl ? 16 : 8;
    const size_t elems = (size_t)batch * ((size_t)M * M + 2 * (size_t)M * K);
    void *buf;
    gw_status s = gwp::ws(ctx, "tune", elems * esz, &buf);
    if (s != GW_OK) return s;
    GW_HIP(ctx, gwk::launch_fill_u32(st, (uint32_t *)buf, (int64_t)(elems * esz / 4), 0u));
    hipEvent_t e0, e1;
    GW_HIP(ctx, hipEventCreate(&e0));
    GW_HIP(ctx, hipEventCreate(&e1));
    auto launch = [&]() -> hipError_t {
        if (dbl) {
            gwk::zdbl *C = (gwk::zdbl *)buf, *A = C + (size_t)batch * M * M, *B = A + (size_t)batch * M * K;
            return gwk::launch_zgemm_lu(st, M, M, K, -1.0, A, K, (int64_t)M * K, B, M, (int64_t)K * M, 1.0, C, M,
                                        (int64_t)M * M, batch);
        }
        gwk::zflt *C = (gwk::zflt *)buf, *A = C + (size_t)batch * M * M, *B = A + (size_t)batch * M * K;
        return gwk::launch_cgemm(st, M, M, K, -1.f, A, K, (int64_t)M * K, B, M, (int64_t)K * M, 1.f, C, M,
                                 (int64_t)M * M, batch);
    };
    double best = 1e300;
    int best_t = 3;
    gwp::Bf16xScope plain(false);  // time the plain complex-float kernel
    for (int t = 3; t >= 0 && s == GW_OK; --t) {
        gwp::set_thread_gemm_tile(t);
        std::vector<double> ms;
        for (int rep = 0; rep < 6; ++rep) {
            hipError_t e = hipEventRecord(e0, st);
            if (e == hipSuccess) e = launch();
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float f = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
            if (e != hipSuccess) {
                s = fail(ctx, GW_E_DEVICE, std::string("autotuner: ") + hipGetErrorString(e));
                break;
            }
            if (rep > 0) ms.push_back(f);  // the first launch warms up
        }
        if (s != GW_OK) break;
        const double med = gwt::median(ms);
        if (med < best) {
            best = med;
            best_t = t;
        }
    }
    gwp::set_thread_gemm_tile(-1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != GW_OK) return s;
    g_tune[key] = best_t;
    std::string err;
    if (!gwt::save(path, g_tune, &err)) ctx->err = "autotuner table not saved: " + err;
    *tile = best_t;
    return GW_OK;
}

void destroy_graph(gw_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Record every molecule's solve program (lock-step mode).  The recording runs
// under a capture of a private stream, so a launch that escaped the recorder
// would land in that throwaway graph instead of running: it is counted and
// refused.
gw_status record_programs(gw_batch *b, std::vector<gwp::SolvePlan> &sp, const std::vector<char> &route_a,
                          std::vector<std::vector<gwk::RecOp>> *progs) {
    gw_ctx *ctx = b->ctx;
    const bool mixed = b->prec != GW_FP64;
    hipStream_t probe = b->branches[0];
    GW_HIP(ctx, hipStreamBeginCapture(probe, hipStreamCaptureModeThreadLocal));
    gw_status s = GW_OK;
    progs->assign(b->n_mol, {});
    {
        gwp::Bf16xScope bf16x(b->prec == GW_BF16X_IR);
        for (int i = 0; i < b->n_mol && s == GW_OK; ++i) {
            gwk::OpRecorder rec;
            gwk::g_rec = &rec;
            gwp::set_thread_gemm_tile(b->tile[i]);
            gwp::zdbl *buf = (gwp::zdbl *)b->chi0[i];
            s = gwp::solve_enqueue_nosync(ctx, sp[i], probe, b->v[i], 0, route_a[i] ? nullptr : buf,
                                          (gwp::zdbl *)b->W[i], mixed ? b->n_refine : 0, route_a[i] ? buf : nullptr);
            gwk::g_rec = nullptr;
            (*progs)[i] = std::move(rec.ops);
        }
        gwp::set_thread_gemm_tile(-1);
    }
    hipGraph_t pg = nullptr;
    const hipError_t e = hipStreamEndCapture(probe, &pg);
    size_t nodes = 0;
    if (pg) {
        (void)hipGraphGetNodes(pg, nullptr, &nodes);
        (void)hipGraphDestroy(pg);
    }
    if (s != GW_OK) return s;
    GW_HIP(ctx, e);
    if (nodes) return fail(ctx, GW_E_DEVICE, "lock step: a solve launch was not recorded");
    return GW_OK;
}

gw_status record(gw_batch *b) {
    gw_ctx *ctx = b->ctx;
    hipStream_t st = b->cap;
    const int nbr = (int)b->branches.size();
    const bool mixed = b->prec != GW_FP64;
    const bool lock = b->mode != 0;
    // planning, pass 1 (grows the shared buffers) and pass 2 (final pointers);
    // lock-stepped molecules all solve at once: a workspace each
    std::vector<gwp::BuildPlan> bp(b->n_mol);
    std::vector<gwp::SolvePlan> sp(b->n_mol);
    // per-molecule workspaces of earlier lock-step batches are reused where
    // they fit; they are released first when keeping them beside this
    // batch's could take more than half the budget (a batch of many small
    // molecules after one of a few large ones would otherwise keep both)
    if (lock) {
        size_t held = 0, need = 0;
        for (auto &kv : ctx->bufs)
            if (kv.first.compare(0, 2, "bl") == 0) held += kv.second.bytes;
        for (int i = 0; i < b->n_mol; ++i)
            need += gwk_solve_ws_bytes(b->n[i], b->g.n_omega, mixed, ctx->budget / b->n_mol);
        if (held + need > ctx->budget / 2) gwp::ws_release(ctx, "bl");
    }
    for (int pass = 0; pass < 2; ++pass) {
        for (int i = 0; i < b->n_mol; ++i) {
            gw_status s = gwp::build_plan(ctx, &b->mols[i], &b->g, nullptr, 0, st, "bb", nullptr, &bp[i]);
            if (s != GW_OK) return s;
            s = lock ? gwp::solve_plan(ctx, b->n[i], b->g.n_omega, mixed, "bl" + std::to_string(i), &sp[i],
                                       ctx->budget / b->n_mol)
                     : gwp::solve_plan(ctx, b->n[i], b->g.n_omega, mixed, "bs" + std::to_string(i % nbr), &sp[i],
                                       ctx->budget / nbr);
            if (s != GW_OK) return s;
            sp[i].final_norms = b->norms[i];
        }
    }
    // in-place molecules never expose chi0: they take the route that forms
    // A = 1 - v chi0 from v a0 in the buffer (one real product per bin instead
    // of one complex product per solved frequency); the builds run one after
    // another on the capture stream, so they share one workspace
    std::vector<char> route_a(b->n_mol, 0);
    std::vector<gwp::ARouteWs> aw(b->n_mol);
    const bool mesh_a = gwp::a_mesh_ok(b->g.n_omega);
    for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i < b->n_mol; ++i) {
            route_a[i] = mesh_a && b->W[i] == b->chi0[i];
            if (!route_a[i]) continue;
            gw_status s = gwp::a_route_ws(ctx, "ba", b->n[i], bp[i].nhb, b->g.n_omega, &aw[i]);
            if (s != GW_OK) return s;
        }
    gwp::LockStep *ls = nullptr;
    if (lock) {
        std::vector<std::vector<gwk::RecOp>> progs;
        gw_status s = record_programs(b, sp, route_a, &progs);
        if (s == GW_OK) s = gwp::lockstep_plan(ctx, std::move(progs), b->mode == 1, &ls);
        if (s != GW_OK) return s;
        b->ls_stats = gwp::lockstep_stats(ls);
    }
    struct Free {
        gwp::LockStep *p;
        ~Free() {
            if (p) gwp::lockstep_free(p);
        }
    } free_ls{ls};
    GW_HIP(ctx, hipStreamSynchronize(st));
    GW_HIP(ctx, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    // from here on every failure still ends the capture below
    gw_status s = GW_OK;
    auto hip = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && s == GW_OK) s = fail(ctx, GW_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    for (int i = 0; i < b->n_mol && s == GW_OK; ++i)
        s = route_a[i] ? gwp::a_route_enqueue(ctx, bp[i], st, b->v[i], aw[i], i == 0, b->chi0[i])
                       : gwp::build_enqueue(ctx, bp[i], st, b->chi0[i], i == 0);
    if (s == GW_OK && lock) {
        s = gwp::lockstep_enqueue(ctx, *ls, st, b->branches, b->events);
    } else if (s == GW_OK) {
        hip(hipEventRecord(b->events[0], st), "fork");
        for (int r = 0; r < nbr; ++r) hip(hipStreamWaitEvent(b->branches[r], b->events[0], 0), "fork");
        gwp::Bf16xScope bf16x(b->prec == GW_BF16X_IR);
        for (int i = 0; i < b->n_mol && s == GW_OK; ++i) {
            gwp::set_thread_gemm_tile(b->tile[i]);
            gwp::zdbl *buf = (gwp::zdbl *)b->chi0[i];
            s = gwp::solve_enqueue_nosync(ctx, sp[i], b->branches[i % nbr], b->v[i], 0, route_a[i] ? nullptr : buf,
                                          (gwp::zdbl *)b->W[i], mixed ? b->n_refine : 0, route_a[i] ? buf : nullptr);
        }
        gwp::set_thread_gemm_tile(-1);
        for (int r = 0; r < nbr; ++r) {
            hip(hipEventRecord(b->events[1 + r], b->branches[r]), "join");
            hip(hipStreamWaitEvent(st, b->events[1 + r], 0), "join");
        }
    }
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(st, &graph);
    if (s != GW_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    GW_HIP(ctx, e);
    b->graph = graph;
    GW_HIP(ctx, hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0));
    return GW_OK;
}

}  // namespace

extern "C" {

gw_status gw_batch_create(gw_ctx *ctx, int32_t n_mol, const gw_molecule *mols, const double *const *v,
                          const gw_grid *g, gw_precision prec, double tol, int32_t n_refine, void *stream,
                          void *const *chi0_out, void *const *W_out, gw_batch **out) {
    if (!ctx || !out) return GW_E_INVALID;
    *out = nullptr;
    if (ctx->sticky) return fail(ctx, GW_E_DEVICE, "context has a sticky device error: " + ctx->err);
    if (n_mol < 1 || !mols || !v || !g || !chi0_out || !W_out) return fail(ctx, GW_E_INVALID, "bad batch arguments");
    if (prec != GW_FP64 && prec != GW_FP32_IR && prec != GW_BF16X_IR)
        return fail(ctx, GW_E_INVALID, "unknown batch precision");
    if (prec != GW_FP64 && (n_refine < 1 || n_refine > 6 || !(tol > 0)))
        return fail(ctx, GW_E_INVALID, "mixed batch needs 1..6 refinement steps and tol > 0");
    for (int i = 0; i < n_mol; ++i)
        if (!v[i] || !chi0_out[i] || !W_out[i]) return fail(ctx, GW_E_INVALID, "NULL buffer in batch");
    GW_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    gw_batch *b = new gw_batch();
    b->ctx = ctx;
    b->n_mol = n_mol;
    b->mols.assign(mols, mols + n_mol);
    b->v.assign(v, v + n_mol);
    b->chi0.assign(chi0_out, chi0_out + n_mol);
    b->W.assign(W_out, W_out + n_mol);
    b->g = *g;
    b->prec = prec;
    b->tol = tol;
    b->n_refine = n_refine;
    if (const char *e = std::getenv("GW_BATCH_MODE")) {
        const std::string m = e;
        if (m == "streams") b->mode = 0;
        else if (m == "lockstep") b->mode = 1;
        else if (m == "lockstep_left") b->mode = 2;
        else {
            delete b;
            return fail(ctx, GW_E_INVALID, "GW_BATCH_MODE must be streams, lockstep or lockstep_left");
        }
    }
    int nbr = 4;
    if (const char *e = std::getenv("GW_BATCH_STREAMS")) nbr = std::max(1, std::min(16, std::atoi(e)));
    if (b->mode == 0) nbr = std::min(nbr, n_mol);
    auto bail = [&](gw_status s) {
        gw_batch_destroy(b);
        return s;
    };
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(ctx, GW_E_DEVICE, "cannot create batch stream"));
    for (int r = 0; r < nbr; ++r) {
        hipStream_t s2;
        if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(ctx, GW_E_DEVICE, "cannot create batch stream"));
        b->branches.push_back(s2);
    }
    for (int r = 0; r < nbr + 1; ++r) {
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
            return bail(fail(ctx, GW_E_DEVICE, "cannot create batch event"));
        b->events.push_back(ev);
    }
    for (int i = 0; i < n_mol; ++i) {
        b->n.push_back(mols[i].n_prod);
        void *p;
        gw_status s = gwp::ws(ctx, "bnorm" + std::to_string(i), (size_t)g->n_omega * 32, &p);
        if (s != GW_OK) return bail(s);
        b->norms.push_back((double *)p);
        int tile = 0;
        s = tune_tile(ctx, mols[i].n_prod, prec, st, &tile);
        if (s != GW_OK) return bail(s);
        b->tile.push_back(tile);
    }
    // a new batch may grow the shared batch workspaces: older graphs are retired
    b->generation = ++ctx->batch_generation;
    // the caller's stream may hold work on these buffers: finish it first
    GW_HIP(ctx, hipStreamSynchronize(st));
    gw_status s = record(b);
    if (s != GW_OK) return bail(s);
    *out = b;
    return GW_OK;
}

gw_status gw_batch_run(gw_batch *b, void *stream, gw_report *reps) {
    if (!b) return GW_E_INVALID;
    gw_ctx *ctx = b->ctx;
    if (ctx->sticky) return fail(ctx, GW_E_DEVICE, "context has a sticky device error: " + ctx->err);
    GW_HIP(ctx, hipSetDevice(ctx->device));
    if (b->generation != ctx->batch_generation)
        return fail(ctx, GW_E_STATE, "batch was recorded before a newer gw_batch_create on this context; recreate it");
    hipStream_t st = (hipStream_t)stream;
    ctx->ks_n = 0;  // the graph rewrites the context's kernel-spectrum buffer
    GW_HIP(ctx, hipGraphLaunch(b->exec, st));
    const bool mixed = b->prec != GW_FP64;
    if (!mixed && !reps) return GW_OK;
    GW_HIP(ctx, hipStreamSynchronize(st));
    const int N = b->g.n_omega;
    gw_status result = GW_OK;
    for (int i = 0; i < b->n_mol; ++i) {
        int fallback = 0, solved = 0;
        double worst = 0;
        const bool in_place = b->W[i] == b->chi0[i];
        if (mixed) {
            std::vector<double> hn(4 * (size_t)N);
            GW_HIP(ctx, hipMemcpy(hn.data(), b->norms[i], sizeof(double) * 4 * N, hipMemcpyDeviceToHost));
            gwp::SolvePlan p64;
            bool planned = false;
            const int64_t nn = (int64_t)b->n[i] * b->n[i];
            std::vector<int> js;
            js.push_back(0);
            for (int j = N / 2; j < N; ++j) js.push_back(j);
            for (int j : js) {
                ++solved;
                const double dn = std::sqrt(hn[2 * j]), wn = std::sqrt(hn[2 * j + 1]);
                const double dprev = b->n_refine >= 2 ? std::sqrt(hn[2 * (size_t)N + 2 * j]) : wn;
                const double r = dn / std::max(wn, 1e-300);
                if (gwp::ir_converged(b->n_refine, dn, dprev, wn, b->tol)) {
                    worst = std::max(worst, r);
                    continue;
                }
                if (in_place) {
                    // chi0 was overwritten: no FP64 re-solve possible
                    worst = std::max(worst, r);
                    if (result == GW_OK)
                        result = fail(ctx, GW_E_NOCONV,
                                      "batched in-place solve: molecule " + std::to_string(i) + " frequency " +
                                          std::to_string(j) + " did not reach the tolerance");
                    continue;
                }
                if (!planned) {
                    gw_status s = gwp::solve_plan(ctx, b->n[i], 2, false, "bfb", &p64);
                    if (s != GW_OK) return s;
                    planned = true;
                }
                gw_status s = gwp::solve_batch_fp64(ctx, st, b->n[i], b->v[i], 0,
                                                    (const gwp::zdbl *)b->chi0[i] + j * nn,
                                                    (gwp::zdbl *)b->W[i] + j * nn, 1, p64.w);
                if (s != GW_OK) return s;
                ++fallback;
            }
            if (fallback) {
                GW_HIP(ctx, gwk::launch_conj_mirror(st, nn, N, (gwp::zdbl *)b->W[i]));
                GW_HIP(ctx, hipStreamSynchronize(st));
            }
        } else {
            solved = N / 2 + 1;
        }
        if (reps) {
            gw_report &r = reps[i];
            r = gw_report{};
            r.n_solved = solved;
            r.n_fallback = fallback;
            r.max_iter = mixed ? b->n_refine : 0;
            r.max_rel_update = worst;
        }
    }
    return result;
}

gw_status gw_batch_stats(const gw_batch *b, int32_t *mode, int64_t *n_steps, int64_t *n_launches,
                         int64_t *n_products) {
    if (!b) return GW_E_INVALID;
    if (mode) *mode = b->mode;
    if (n_steps) *n_steps = b->ls_stats.steps;
    if (n_launches) *n_launches = b->ls_stats.launches;
    if (n_products) *n_products = b->ls_stats.products;
    return GW_OK;
}

gw_status gw_batch_destroy(gw_batch *b) {
    if (!b) return GW_E_INVALID;
    (void)hipSetDevice(b->ctx->device);
    destroy_graph(b);
    for (auto s : b->branches) (void)hipStreamDestroy(s);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (auto e : b->events) (void)hipEventDestroy(e);
    delete b;
    return GW_OK;
}

}  // extern "C"
