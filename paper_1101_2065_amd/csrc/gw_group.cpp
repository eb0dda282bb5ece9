// Lock-step execution of the batched W solves.
//
// Every molecule's solve program (its frequency batches: LU factorisations,
// substitutions, refinement steps) is recorded as a list of operations by the
// same launchers that run the single-molecule path (a recorder installed on
// the host thread turns their launches into descriptors).  The programs then
// advance together, one operation per molecule per lock step:
//   * all complex products of a lock step are one launch per tile shape over
//     the tiles of every (molecule, frequency, LU step) product in it, either
//     one workgroup per tile handed out by the hardware dispatcher (the
//     default) or, with GW_GEMM_QUEUE=persistent, a persistent grid (as many
//     workgroups as stay resident) pulling tiles from eight per-XCD device
//     counters and stealing from the other seven when theirs runs dry;
//   * all panel factorisations of a lock step are one grouped launch per
//     panel variant, all row exchanges one grouped launch;
//   * anything else (permutations, right-hand sides, mirrors, conversions,
//     norms, split-BF16 products) runs as its own launch in the step.
// Launches of one lock step are independent (different molecules).  In the
// recorded graph each launch depends only on the launches that held the
// previous operations of its own molecules (without a graph capture: the
// launches of a step go to parallel branches and join before the next
// step).  Descriptor tables are uploaded before graph capture, the queue
// counters (persistent form) cleared by one fill kernel at the start of the
// recorded work, so the whole program is one hipGraph.
#include "gw_plan.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <map>
#include <string>
#include <vector>

namespace gwp {

namespace {

struct Launch {
    gwk::RecOp::Kind kind;
    int key = 0;
    int64_t off = 0;  // first descriptor in the device table of its kind
    int n_items = 0;
    int64_t work = 0;  // tiles (products) or workgroups (panels, exchanges)
    int grid = 0;      // products: workgroups of the persistent grid
    int queue = 0;     // products: index of its eight counters
    double flops = 0;
    const gwk::RecOp *op = nullptr;  // OTHER: the deferred launch
    std::vector<int> mols;           // the molecules whose operations it holds
};

}  // namespace

struct LockStep {
    std::vector<std::vector<gwk::RecOp>> progs;
    std::vector<std::vector<Launch>> steps;
    gwk::GemmItem *d_gemm = nullptr;
    gwk::PanelItem *d_panel = nullptr;
    unsigned *d_queue = nullptr;
    int n_queues = 0;
    bool persistent = false;  // products on the persistent work-queue grid
    LockStepStats stats;
    int n_mol = 0;
};

void lockstep_free(LockStep *ls) { delete ls; }

const LockStepStats &lockstep_stats(const LockStep *ls) { return ls->stats; }

gw_status lockstep_plan(gw_ctx *c, std::vector<std::vector<gwk::RecOp>> progs, bool right_align, LockStep **out) {
    *out = nullptr;
    LockStep *ls = new LockStep();
    if (const char *q = std::getenv("GW_GEMM_QUEUE")) ls->persistent = std::string(q) == "persistent";
    for (auto &p : progs) {
        std::vector<gwk::RecOp> q;
        q.reserve(p.size());
        for (auto &o : p)
            if (o.kind != gwk::RecOp::MARK) q.push_back(std::move(o));
        ls->progs.push_back(std::move(q));
    }
    int n_cu = 0;
    hipError_t e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c->device);
    if (e != hipSuccess || n_cu <= 0) {
        delete ls;
        return fail(c, GW_E_DEVICE, "lock step: cannot read the compute-unit count");
    }
    size_t L = 0;
    for (auto &p : ls->progs) L = std::max(L, p.size());
    const int nm = (int)ls->progs.size();
    ls->n_mol = nm;
    std::vector<gwk::GemmItem> gi;
    std::vector<gwk::PanelItem> pi;
    std::map<int, int> occ;  // per product key
    auto occupancy = [&](int key) {
        auto it = occ.find(key);
        if (it == occ.end()) it = occ.emplace(key, gwk::gemm_queue_occupancy(key)).first;
        return it->second;
    };
    // Merging couples the molecules of a launch (each waits for the others'
    // previous operations), so only what cannot fill the GPU alone is merged:
    // products of fewer than merge_waves times the resident workgroups, and
    // (merge_panels) panels and row exchanges.
    double merge_waves = 1.0;
    bool merge_panels = false;
    if (const char *e = std::getenv("GW_LOCKSTEP_MERGE_WAVES")) merge_waves = std::atof(e);
    if (const char *e = std::getenv("GW_LOCKSTEP_MERGE_PANELS")) merge_panels = std::atoi(e) != 0;
    ls->steps.resize(L);
    for (size_t k = 0; k < L; ++k) {
        // keys: merged launches by product / panel key; a launch of its own
        // for an operation that is not merged (key + 1000 (1 + molecule))
        std::map<int, std::vector<const gwk::RecOp *>> gemm, panel, laswp;
        std::vector<const gwk::RecOp *> other;
        std::map<const gwk::RecOp *, int> owner;
        for (int i = 0; i < nm; ++i) {
            const auto &p = ls->progs[i];
            const size_t off = right_align ? L - p.size() : 0;
            if (k < off || k - off >= p.size()) continue;
            const gwk::RecOp &o = p[k - off];
            owner[&o] = i;
            const int own = 1000 * (1 + i);
            if (o.kind == gwk::RecOp::GEMM) {
                int bm = 0, bn = 0;
                gwk::gemm_queue_tile(o.key, &bm, &bn);
                const double tiles = (double)((o.g.M + bm - 1) / bm) * ((o.g.N + bn - 1) / bn) * o.g.batch;
                const bool merge = tiles < merge_waves * n_cu * occupancy(o.key);
                gemm[o.key + (merge ? 0 : own)].push_back(&o);
            } else if (o.kind == gwk::RecOp::PANEL) {
                panel[o.key + (merge_panels ? 0 : own)].push_back(&o);
            } else if (o.kind == gwk::RecOp::LASWP) {
                laswp[o.key + (merge_panels ? 0 : own)].push_back(&o);
            } else {
                other.push_back(&o);
            }
        }
        // latency-bound launches (panels, row exchanges, the rest: few
        // workgroups) first, so that they hold their compute units before the
        // persistent product grid fills the others
        auto &st = ls->steps[k];
        auto grouped = [&](std::map<int, std::vector<const gwk::RecOp *>> &m, gwk::RecOp::Kind kind) {
            for (auto &kv : m) {
                Launch l;
                l.kind = kind;
                l.key = kv.first % 1000;
                l.off = (int64_t)pi.size();
                int64_t wg = 0;
                for (const gwk::RecOp *o : kv.second) {
                    gwk::PanelItem p = o->p;
                    p.wg0 = wg;
                    wg += kind == gwk::RecOp::PANEL ? (int64_t)p.batch
                                                    : (int64_t)p.batch * ((p.n - p.w + 31) / 32);
                    pi.push_back(p);
                    l.mols.push_back(owner[o]);
                }
                l.n_items = (int)kv.second.size();
                l.work = wg;
                st.push_back(l);
            }
        };
        grouped(panel, gwk::RecOp::PANEL);
        grouped(laswp, gwk::RecOp::LASWP);
        for (const gwk::RecOp *o : other) {
            Launch l;
            l.kind = gwk::RecOp::OTHER;
            l.op = o;
            l.mols.push_back(owner[o]);
            st.push_back(l);
        }
        for (auto &kv : gemm) {
            Launch l;
            l.kind = gwk::RecOp::GEMM;
            l.key = kv.first % 1000;
            l.off = (int64_t)gi.size();
            int bm = 0, bn = 0;
            gwk::gemm_queue_tile(l.key, &bm, &bn);
            int64_t t = 0;
            for (const gwk::RecOp *o : kv.second) {
                gwk::GemmItem g = o->g;
                g.tx = (g.N + bn - 1) / bn;
                g.ty = (g.M + bm - 1) / bm;
                g.t0 = t;
                t += (int64_t)g.tx * g.ty * g.batch;
                gi.push_back(g);
                l.flops += o->flops;
                l.mols.push_back(owner[o]);
            }
            l.n_items = (int)kv.second.size();
            l.work = t;
            l.grid = (int)std::min<int64_t>(t, (int64_t)n_cu * occupancy(l.key));
            if (ls->persistent) l.queue = ls->n_queues++;
            ls->stats.products += l.n_items;
            st.push_back(l);
        }
        ls->stats.launches += (int64_t)st.size();
    }
    ls->stats.steps = (int64_t)L;
    for (auto &p : ls->progs) ls->stats.ops += (int64_t)p.size();
    // device tables (uploaded now: nothing is copied while the graph records)
    void *q;
    gw_status s = GW_OK;
    if ((s = ws(c, "lsGemm", std::max<size_t>(1, gi.size()) * sizeof(gwk::GemmItem), &q)) == GW_OK) {
        ls->d_gemm = (gwk::GemmItem *)q;
        if ((s = ws(c, "lsPanel", std::max<size_t>(1, pi.size()) * sizeof(gwk::PanelItem), &q)) == GW_OK) {
            ls->d_panel = (gwk::PanelItem *)q;
            if ((s = ws(c, "lsQueue", std::max<size_t>(1, (size_t)ls->n_queues * 8) * sizeof(unsigned), &q)) == GW_OK)
                ls->d_queue = (unsigned *)q;
        }
    }
    if (s != GW_OK) {
        delete ls;
        return s;
    }
    e = hipSuccess;
    if (!gi.empty()) e = hipMemcpy(ls->d_gemm, gi.data(), gi.size() * sizeof(gwk::GemmItem), hipMemcpyHostToDevice);
    if (e == hipSuccess && !pi.empty())
        e = hipMemcpy(ls->d_panel, pi.data(), pi.size() * sizeof(gwk::PanelItem), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        delete ls;
        return fail(c, GW_E_DEVICE, std::string("lock step: descriptor upload: ") + hipGetErrorString(e));
    }
    *out = ls;
    return GW_OK;
}

gw_status lockstep_enqueue(gw_ctx *c, const LockStep &ls, hipStream_t st, const std::vector<hipStream_t> &branches,
                           const std::vector<hipEvent_t> &events) {
    if (branches.empty() || events.size() < branches.size() + 1)
        return fail(c, GW_E_INVALID, "lock step: needs branches and their events");
    const int nb = (int)branches.size();
    if (ls.n_queues > 0) GW_HIP(c, gwk::launch_fill_u32(st, ls.d_queue, (int64_t)ls.n_queues * 8, 0u));
    auto run = [&](const Launch &l, hipStream_t s) -> hipError_t {
        switch (l.kind) {
            case gwk::RecOp::GEMM:
                return gwk::launch_gemm_queue(s, l.key, ls.d_gemm + l.off, l.n_items, l.work,
                                              ls.persistent ? ls.d_queue + 8 * l.queue : nullptr, l.grid, l.flops);
            case gwk::RecOp::PANEL:
                return gwk::launch_panel_group(s, l.key, ls.d_panel + l.off, l.n_items, l.work);
            case gwk::RecOp::LASWP:
                return gwk::launch_laswp_group(s, l.key, ls.d_panel + l.off, l.n_items, l.work);
            default:
                return l.op->fn(s);
        }
    };
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    GW_HIP(c, hipStreamIsCapturing(st, &cs));
    const char *dm = std::getenv("GW_LOCKSTEP_DEPS");
    if (cs == hipStreamCaptureStatusActive && !(dm && std::string(dm) == "step")) {
        // Recorded with exact dependencies: each launch waits for the
        // launches that held the previous operation of each of its molecules,
        // nothing else, so a molecule whose launch is short runs ahead
        // instead of waiting for the whole step.  All launches are captured
        // on st with the stream's dependency set replaced before each.
        auto terminal = [&](std::vector<hipGraphNode_t> *out) -> hipError_t {
            hipStreamCaptureStatus s2;
            const hipGraphNode_t *d = nullptr;
            size_t nd = 0;
            hipError_t e = hipStreamGetCaptureInfo_v2(st, &s2, nullptr, nullptr, &d, &nd);
            if (e == hipSuccess) out->assign(d, d + nd);
            return e;
        };
        std::vector<hipGraphNode_t> base;
        GW_HIP(c, terminal(&base));
        std::vector<std::vector<hipGraphNode_t>> last(ls.n_mol, base);
        std::vector<hipGraphNode_t> deps, after;
        for (const auto &step : ls.steps)
            for (const Launch &l : step) {
                deps.clear();
                for (int i : l.mols) deps.insert(deps.end(), last[i].begin(), last[i].end());
                std::sort(deps.begin(), deps.end());
                deps.erase(std::unique(deps.begin(), deps.end()), deps.end());
                GW_HIP(c, hipStreamUpdateCaptureDependencies(st, deps.data(), deps.size(),
                                                             hipStreamSetCaptureDependencies));
                GW_HIP(c, run(l, st));
                GW_HIP(c, terminal(&after));
                for (int i : l.mols) last[i] = after;
            }
        // whatever follows waits for every molecule's last launch
        deps.clear();
        for (auto &v : last) deps.insert(deps.end(), v.begin(), v.end());
        std::sort(deps.begin(), deps.end());
        deps.erase(std::unique(deps.begin(), deps.end()), deps.end());
        GW_HIP(c, hipStreamUpdateCaptureDependencies(st, deps.data(), deps.size(), hipStreamSetCaptureDependencies));
        return GW_OK;
    }
    // step by step: the launches of a step on parallel branches (the first on
    // the main stream), joined before the next step
    for (const auto &step : ls.steps) {
        if (step.empty()) continue;
        if (step.size() == 1) {
            GW_HIP(c, run(step[0], st));
            continue;
        }
        const int used = std::min<int>(nb, (int)step.size() - 1);
        GW_HIP(c, hipEventRecord(events[0], st));
        for (int r = 0; r < used; ++r) GW_HIP(c, hipStreamWaitEvent(branches[r], events[0], 0));
        GW_HIP(c, run(step[0], st));
        for (size_t j = 1; j < step.size(); ++j) GW_HIP(c, run(step[j], branches[(j - 1) % nb]));
        for (int r = 0; r < used; ++r) {
            GW_HIP(c, hipEventRecord(events[1 + r], branches[r]));
            GW_HIP(c, hipStreamWaitEvent(st, events[1 + r], 0));
        }
    }
    return GW_OK;
}

}  // namespace gwp
