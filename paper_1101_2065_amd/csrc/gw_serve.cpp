// Serving: continuous batching of molecule solves on one GPU.
//
// gw_submit queues a request and returns a ticket at once.  A fixed number of
// slots (GW_SERVE_SLOTS, default 2) each own a host thread, a HIP stream and a
// private context.  A free slot admits the request at the head of the queue
// as soon as its estimated HBM footprint (workspace + results) fits under the
// context's budget, next to the results still held and the workspace the
// other slots keep; admitted requests run concurrently on their slots'
// streams, so work of different molecules overlaps on the device: the
// compression and A build of one request (vector units, HBM) run beside
// the W solve of another (matrix cores).  The solves themselves take turns
// (GW_SERVE_SOLVE_OVERLAP=1 lets them run together): the LU panel kernel needs
// a whole CU, which a concurrent solve's GEMM workgroups keep occupied.  All
// serving memory is stream-ordered (hipMallocAsync / hipFreeAsync on the
// slot's stream, recycled by the device pool), so no allocation or release
// synchronises the device.  A slot keeps its workspace for the next request
// and only gives it back when the head of the queue would not fit otherwise;
// the results (W, plus the compression basis) stay resident until
// gw_release; A = 1 - v chi0 is formed in W's buffer and solved there, so
// chi0 itself is never held (GW_SERVE_CHI0=1 forms it in a buffer of its own).  Requests are admitted in arrival order; gw_release on a request
// still in the queue cancels it.  A request that runs out of device memory
// (others' results and workspace in the way) goes back to the head of the
// queue once, after its slot has given back its workspace.
#include "../../include/gw.h"
#include "gw_ctx.h"
#include "gw_internal.h"
#include "gw_plan.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <condition_variable>
#include <cstdlib>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace {

enum ReqState { Q_QUEUED, Q_RUNNING, Q_DONE, Q_FAILED };

struct ServeReq {
    uint64_t ticket = 0;
    gw_molecule mol{};
    const double *v = nullptr;
    gw_grid grid{};
    int k = 0, kk = 0;
    bool route_a = true;  // A formed in W's buffer and solved in place (else chi0 first)
    gw_precision prec = GW_FP64;
    double tol = 1e-7;
    size_t bytes_result = 0, bytes_ws = 0, bytes_peak = 0;
    ReqState state = Q_QUEUED;
    void *chi = nullptr, *res = nullptr, *Q = nullptr, *S = nullptr;
    hipStream_t stream = nullptr;  // the slot stream its buffers were allocated on
    gw_report rep{};
    gw_status status = GW_OK;
    std::string err;
    int retries = 0;  // times it went back to the queue after running out of memory
};

}  // namespace

struct GwServe {
    std::mutex mu;
    std::mutex solve_mu;  // one W solve on the device at a time
    std::condition_variable cv;
    std::deque<uint64_t> queue;
    std::map<uint64_t, std::unique_ptr<ServeReq>> reqs;
    size_t budget = 0;
    size_t results = 0;        // result buffers of running and finished, unreleased requests
    std::vector<size_t> held;  // workspace each slot keeps between requests
    size_t slot_ws_budget = 0;
    std::vector<std::thread> workers;
    bool stop = false;
    uint64_t next_ticket = 1;
    int device = 0;
};

namespace {

size_t est_transient(const gw_molecule &m, int k, int n_omega, gw_precision prec, size_t slot_budget,
                     bool route_a) {
    const size_t n_prod = m.n_prod, n_occ = m.n_occ, n_virt = m.n_orb - m.n_occ;
    const size_t n_pairs = n_occ * n_virt;
    const size_t kk = k ? (size_t)k : n_prod;
    const size_t nhb = n_omega / 2;
    size_t b = 0;
    if (route_a) {
        b += 8 * nhb * kk * kk;                                        // v a0 per bin
        b += std::min<size_t>(2ull << 30, 8 * kk * kk * nhb);          // staged dense bins
        b += 16 * (nhb + 1) * nhb;                                     // Cauchy matrix
    }
    if (k) {
        const size_t chunk_rows = std::max<size_t>(1, (size_t)(2ull << 30) / (8 * n_prod * n_virt));
        b += 8 * n_prod * std::min(n_occ, chunk_rows) * n_virt;  // pair-vector chunk
        b += 8 * kk * n_pairs;                                   // projected pair vectors
        b += 8 * (size_t)k * n_prod;                             // basis transpose
        b += 8 * gwk::compress_work_doubles((int)n_prod, k);     // basis iteration
    } else {
        b += 8 * n_prod * n_pairs;
    }
    b += 8 * kk * n_pairs;                                       // bin-sorted pair vectors
    b += 4 * n_occ * (2 * nhb + 1) + 4 * nhb + 12 * n_pairs + 4096;
    b += 8 * nhb * kk * (kk + 1) / 2;                            // histogram
    b += 2 * 16 * 2 * (size_t)n_omega;                           // kernel spectrum, twiddles
    b += gwk_solve_ws_bytes((int)kk, n_omega, prec != GW_FP64, slot_budget);
    return b + (64ull << 20);
}

// GW_SERVE_TRACE=1: one line per request on stderr with its phase times.
bool trace_on() {
    static const bool on = [] {
        const char *e = std::getenv("GW_SERVE_TRACE");
        return e && *e && *e != '0';
    }();
    return on;
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool solve_overlap() {
    static const bool on = [] {
        const char *e = std::getenv("GW_SERVE_SOLVE_OVERLAP");
        return e && *e && *e != '0';
    }();
    return on;
}

void run_request(gw_ctx *child, hipStream_t st, ServeReq &r, std::mutex *solve_mu) {
    const bool tr = trace_on();
    double t[6] = {now_ms(), 0, 0, 0, 0, 0};
    auto mark = [&](int i) {
        if (!tr) return;
        (void)hipStreamSynchronize(st);
        t[i] = now_ms();
    };
    struct Report {
        bool on;
        double *t;
        ServeReq &r;
        ~Report() {
            if (on)
                std::fprintf(stderr, "gw serve: ticket %llu n_prod %d k %d basis %.1f alloc %.1f chi0 %.1f solve %.1f "
                                     "total %.1f ms\n",
                             (unsigned long long)r.ticket, r.mol.n_prod, r.k, t[1] - t[0], t[2] - t[1], t[3] - t[2],
                             t[4] - t[3], now_ms() - t[0]);
        }
    } report{tr, t, r};
    auto hip_ok = [&](hipError_t e, const char *what) {
        if (e == hipSuccess) return true;
        r.status = e == hipErrorOutOfMemory ? GW_E_OOM : GW_E_DEVICE;
        r.err = std::string(what) + ": " + hipGetErrorString(e);
        return false;
    };
    const size_t nn = (size_t)r.kk * r.kk;
    const size_t n = r.mol.n_prod;
    if (r.k) {
        if (!hip_ok(gwk_malloc_async((void **)&r.Q, 8 * n * r.k, st), "basis")) return;
        if (!hip_ok(gwk_malloc_async((void **)&r.S, 8 * (size_t)r.k * r.k, st), "metric")) return;
        gw_status s = gw_compress_basis(child, r.v, (int)n, r.k, st, (double *)r.Q, (double *)r.S);
        if (s != GW_OK) {
            r.status = s;
            r.err = gw_last_error(child);
            return;
        }
    }
    mark(1);
    // chi0 is returned to nobody: A = 1 - v chi0 (compressed: 1 - S chi_hat)
    // is formed from v a0 in W's buffer and solved there in place; only a
    // mesh the FFT form of the transform cannot take goes through chi0
    if (!r.route_a && !hip_ok(gwk_malloc_async((void **)&r.chi, 16 * nn * r.grid.n_omega, st), "chi0")) return;
    const size_t res_bytes = 16 * nn * r.grid.n_omega + (r.k ? 8 * n * r.k : 0);
    if (!hip_ok(gwk_malloc_async((void **)&r.res, res_bytes, st), "W")) return;
    mark(2);
    gw_report rb{}, rs{};
    const double *vk = r.k ? (const double *)r.S : r.v;
    gw_status s;
    if (!r.route_a)
        s = gw_build_chi0(child, &r.mol, &r.grid, (const double *)r.Q, r.k, st, nullptr, r.chi, &rb);
    else if (r.k)
        s = gw_build_A_compressed(child, &r.mol, vk, (const double *)r.Q, r.k, &r.grid, st, r.res, &rb);
    else
        s = gw_build_A(child, &r.mol, r.v, &r.grid, st, r.res, &rb);
    mark(3);
    if (s == GW_OK) {
        // the solve returns after its stream has drained (it reports), so
        // holding the lock across it keeps the solves apart on the device
        std::unique_lock<std::mutex> lk(*solve_mu, std::defer_lock);
        if (!solve_overlap()) lk.lock();
        if (r.route_a)
            s = gw_solve_W_A(child, vk, 0, r.kk, r.res, r.grid.n_omega, r.prec, r.tol, st, r.res, &rs);
        else
            s = gw_solve_W(child, vk, 0, r.kk, r.chi, r.grid.n_omega, r.prec, r.tol, st, r.res, &rs);
    }
    if (s != GW_OK) {
        r.status = s;
        r.err = gw_last_error(child);
        return;
    }
    if (r.k) {
        char *tail = (char *)r.res + 16 * nn * r.grid.n_omega;
        if (!hip_ok(hipMemcpyAsync(tail, r.Q, 8 * n * r.k, hipMemcpyDeviceToDevice, st), "copy basis")) return;
    }
    if (!hip_ok(hipStreamSynchronize(st), "stream")) return;
    mark(4);
    r.rep = rs;
    r.rep.n_hbins = rb.n_hbins;
    r.rep.frac_bits_used = rb.frac_bits_used;
    r.rep.n_dropped_pairs = rb.n_dropped_pairs;
}

// Stream-ordered free on the stream that produced the buffers (no device-wide
// synchronisation; the memory goes back to the device's pool).
void free_results(ServeReq &r) {
    for (void **p : {&r.chi, &r.res, &r.Q, &r.S})
        if (*p) {
            (void)hipFreeAsync(*p, r.stream);
            *p = nullptr;
        }
}

// Can slot i admit h?  Results in use, every other slot's kept workspace and
// this slot's workspace grown to h's estimate must fit the budget.
bool fits(const GwServe *sv, int i, const ServeReq *h) {
    size_t others = 0;
    for (size_t j = 0; j < sv->held.size(); ++j)
        if ((int)j != i) others += sv->held[j];
    return sv->results + h->bytes_result + others + std::max(sv->held[i], h->bytes_ws) <= sv->budget;
}

// One serving slot.  The slot keeps its workspace between requests (no
// allocation churn); it gives it back only when the request at the head of
// the queue would not fit otherwise.
void worker(GwServe *sv, int slot) {
    (void)hipSetDevice(sv->device);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
    gw_ctx *child = nullptr;
    if (gw_create(sv->device, sv->slot_ws_budget, &child) != GW_OK) {
        (void)hipStreamDestroy(st);
        return;
    }
    child->own_stream = st;
    for (;;) {
        ServeReq *r = nullptr;
        bool trim = false;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            for (;;) {
                if (sv->stop) break;
                if (!sv->queue.empty()) {
                    ServeReq *h = sv->reqs[sv->queue.front()].get();
                    if (fits(sv, slot, h)) {
                        r = h;
                        sv->queue.pop_front();
                        sv->results += r->bytes_result;
                        sv->held[slot] = std::max(sv->held[slot], r->bytes_ws);
                        r->state = Q_RUNNING;
                        break;
                    }
                    if (sv->held[slot] > 0) {
                        trim = true;
                        break;
                    }
                }
                sv->cv.wait(lk);
            }
            if (sv->stop) break;
        }
        if (trim) {
            gwk_ctx_trim(child);
            (void)hipStreamSynchronize(st);
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                sv->held[slot] = 0;
            }
            sv->cv.notify_all();
            continue;
        }
        r->stream = st;
        run_request(child, st, *r, &sv->solve_mu);
        // out of memory (other requests' results and workspace in the way):
        // the slot gives its workspace back and the request goes back to the
        // head of the queue, once; a second failure is reported
        const bool retry = r->status == GW_E_OOM && r->retries == 0;
        if (retry) gwk_ctx_trim(child);
        const size_t kept = gwk_ctx_bytes(child);
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->held[slot] = kept;
            if (r->status != GW_OK) {
                free_results(*r);
                sv->results -= r->bytes_result;
                if (retry) {
                    r->retries = 1;
                    r->status = GW_OK;
                    r->err.clear();
                    r->state = Q_QUEUED;
                    sv->queue.push_front(r->ticket);
                } else {
                    r->state = Q_FAILED;
                    if (r->retries) r->err += " (after one retry)";
                }
            } else {
                r->state = Q_DONE;
            }
        }
        sv->cv.notify_all();
    }
    gw_destroy(child);
    (void)hipStreamDestroy(st);
}

GwServe *serve_of(gw_ctx *ctx) {
    if (ctx->serve) return ctx->serve;
    GwServe *sv = new GwServe();
    sv->device = ctx->device;
    // keep memory freed by finished requests in the device pool for the next ones
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, ctx->device) == hipSuccess && pool) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    sv->budget = ctx->budget;
    int slots = 2;
    if (const char *e = std::getenv("GW_SERVE_SLOTS")) slots = std::max(1, std::min(8, std::atoi(e)));
    sv->slot_ws_budget = std::min<size_t>(32ull << 30, ctx->budget / (4 * slots));
    sv->held.assign(slots, 0);
    for (int i = 0; i < slots; ++i) sv->workers.emplace_back(worker, sv, i);
    ctx->serve = sv;
    return sv;
}

}  // namespace

void gwk_serve_stop(gw_ctx *ctx) {
    GwServe *sv = ctx->serve;
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv.notify_all();
    for (auto &t : sv->workers) t.join();
    (void)hipSetDevice(sv->device);
    (void)hipDeviceSynchronize();
    for (auto &kv : sv->reqs)
        for (void **p : {&kv.second->chi, &kv.second->res, &kv.second->Q, &kv.second->S})
            if (*p) {
                (void)hipFree(*p);
                *p = nullptr;
            }
    delete sv;
    ctx->serve = nullptr;
}

extern "C" {

gw_status gw_submit(gw_ctx *ctx, const gw_molecule *m, const double *v, const gw_grid *g, int32_t k_compress,
                    gw_precision prec, double tol, uint64_t *ticket) {
    if (!ctx || !m || !v || !g || !ticket) return GW_E_INVALID;
    if (ctx->sticky) return GW_E_DEVICE;
    if (m->n_prod < 1 || m->n_orb < 2 || m->n_occ < 1 || m->n_occ >= m->n_orb) {
        ctx->err = "gw_submit: bad molecule sizes";
        return GW_E_INVALID;
    }
    if (k_compress < 0 || k_compress > m->n_prod) {
        ctx->err = "gw_submit: k_compress must be in [0, n_prod]";
        return GW_E_INVALID;
    }
    if (prec != GW_FP64 && prec != GW_FP32_IR && prec != GW_BF16X_IR) {
        ctx->err = "gw_submit: precision not available for serving";
        return GW_E_INVALID;
    }
    if (g->n_omega < 16 || g->n_omega > 2048 || (g->n_omega & (g->n_omega - 1))) {
        ctx->err = "gw_submit: n_omega must be a power of two in [16, 2048]";
        return GW_E_INVALID;
    }
    GwServe *sv = serve_of(ctx);
    auto r = std::make_unique<ServeReq>();
    r->mol = *m;
    r->v = v;
    r->grid = *g;
    r->k = k_compress;
    r->kk = k_compress ? k_compress : m->n_prod;
    r->prec = prec;
    r->tol = tol;
    // GW_SERVE_CHI0=1 keeps chi0 in a buffer of its own (the earlier form)
    const char *ec = std::getenv("GW_SERVE_CHI0");
    r->route_a = gwp::a_mesh_ok(g->n_omega) && !(ec && *ec && *ec != '0');
    const size_t nn = (size_t)r->kk * r->kk;
    r->bytes_result = (r->route_a ? 16 : 32) * nn * g->n_omega +
                      (k_compress ? 16ull * m->n_prod * k_compress + 8ull * nn : 0);
    r->bytes_ws = est_transient(*m, k_compress, g->n_omega, prec, sv->slot_ws_budget, r->route_a);
    r->bytes_peak = r->bytes_result + r->bytes_ws;
    if (r->bytes_peak > sv->budget) {
        ctx->err = "gw_submit: request needs " + std::to_string(r->bytes_peak) + " bytes, more than the budget";
        return GW_E_OOM;
    }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        r->ticket = sv->next_ticket++;
        *ticket = r->ticket;
        sv->queue.push_back(r->ticket);
        sv->reqs[r->ticket] = std::move(r);
    }
    sv->cv.notify_all();
    return GW_OK;
}

gw_status gw_poll(gw_ctx *ctx, uint64_t ticket, void **W_dev, gw_report *rep) {
    if (!ctx) return GW_E_INVALID;
    GwServe *sv = ctx->serve;
    if (!sv) {
        ctx->err = "gw_poll: unknown ticket";
        return GW_E_STATE;
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) {
        ctx->err = "gw_poll: unknown ticket";
        return GW_E_STATE;
    }
    ServeReq &r = *it->second;
    if (r.state == Q_QUEUED || r.state == Q_RUNNING) return GW_PENDING;
    if (r.state == Q_FAILED) {
        ctx->err = "request " + std::to_string(ticket) + ": " + r.err;
        return r.status;
    }
    if (W_dev) *W_dev = r.res;
    if (rep) *rep = r.rep;
    return GW_OK;
}

gw_status gw_release(gw_ctx *ctx, uint64_t ticket) {
    if (!ctx) return GW_E_INVALID;
    GwServe *sv = ctx->serve;
    if (!sv) {
        ctx->err = "gw_release: unknown ticket";
        return GW_E_STATE;
    }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->reqs.find(ticket);
        if (it == sv->reqs.end()) {
            ctx->err = "gw_release: unknown ticket";
            return GW_E_STATE;
        }
        ServeReq &r = *it->second;
        if (r.state == Q_RUNNING) {
            ctx->err = "gw_release: request is running";
            return GW_E_STATE;
        }
        if (r.state == Q_QUEUED) {
            // not admitted yet: cancel
            sv->queue.erase(std::find(sv->queue.begin(), sv->queue.end(), ticket));
        }
        if (r.state == Q_DONE) sv->results -= r.bytes_result;
        free_results(r);
        sv->reqs.erase(it);
    }
    sv->cv.notify_all();
    return GW_OK;
}

}  // extern "C"
