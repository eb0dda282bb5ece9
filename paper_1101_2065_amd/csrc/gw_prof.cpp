// Event-pair kernel timing behind gw_profile_begin / gw_profile_read /
// gw_profile_end.
#include "gw_prof.h"

#include "../../include/gw.h"
#include "gw_ctx.h"

#include <cstring>
#include <map>
#include <string>
#include <vector>

namespace gwk {

struct ProfRec {
    std::string cls;
    double flops = 0, bytes = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
};

struct ProfStat {
    int64_t launches = 0;
    double ms = 0, flops = 0, bytes = 0;
};

struct ProfSink {
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> pool;
    std::map<std::string, ProfStat> acc;
    bool failed = false;
};

thread_local ProfSink *g_prof = nullptr;

namespace {

hipEvent_t take(ProfSink *s) {
    if (!s->pool.empty()) {
        hipEvent_t e = s->pool.back();
        s->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Wait for every recorded pair, add it to the sums, recycle the events.
void flush(ProfSink *s) {
    for (auto &r : s->recs) {
        float ms = 0;
        if (r.e1 && hipEventSynchronize(r.e1) == hipSuccess && hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
            ProfStat &a = s->acc[r.cls];
            a.launches += 1;
            a.ms += ms;
            a.flops += r.flops;
            a.bytes += r.bytes;
        } else {
            s->failed = true;
        }
        if (r.e0) s->pool.push_back(r.e0);
        if (r.e1) s->pool.push_back(r.e1);
    }
    s->recs.clear();
}

void destroy(ProfSink *s) {
    flush(s);
    for (hipEvent_t e : s->pool) (void)hipEventDestroy(e);
    delete s;
}

}  // namespace

int prof_begin(ProfSink *s, hipStream_t st, const char *cls, double flops, double bytes) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return -1;
    if (s->recs.size() >= 8192) flush(s);
    ProfRec r;
    r.cls = cls;
    r.flops = flops;
    r.bytes = bytes;
    r.e0 = take(s);
    r.e1 = take(s);
    if (!r.e0 || !r.e1 || hipEventRecord(r.e0, st) != hipSuccess) {
        if (r.e0) s->pool.push_back(r.e0);
        if (r.e1) s->pool.push_back(r.e1);
        s->failed = true;
        return -1;
    }
    s->recs.push_back(r);
    return (int)s->recs.size() - 1;
}

void prof_end(ProfSink *s, hipStream_t st, int slot) {
    if (hipEventRecord(s->recs[slot].e1, st) != hipSuccess) {
        s->pool.push_back(s->recs[slot].e1);
        s->recs[slot].e1 = nullptr;
    }
}

}  // namespace gwk

extern "C" {

gw_status gw_profile_begin(gw_ctx *ctx) {
    if (!ctx) return GW_E_INVALID;
    if (hipSetDevice(ctx->device) != hipSuccess) return GW_E_DEVICE;
    if (!ctx->prof) ctx->prof = new gwk::ProfSink();
    gwk::flush(ctx->prof);
    ctx->prof->acc.clear();
    ctx->prof->failed = false;
    gwk::g_prof = ctx->prof;
    return GW_OK;
}

gw_status gw_profile_read(gw_ctx *ctx, gw_kernel_stat *out, int32_t cap, int32_t *n_out) {
    if (!ctx || !n_out || (cap > 0 && !out)) return GW_E_INVALID;
    *n_out = 0;
    if (!ctx->prof) {
        ctx->err = "gw_profile_read: profiling was not started";
        return GW_E_STATE;
    }
    gwk::flush(ctx->prof);
    int32_t i = 0;
    for (auto &kv : ctx->prof->acc) {
        if (i < cap) {
            gw_kernel_stat &o = out[i];
            std::memset(&o, 0, sizeof(o));
            std::strncpy(o.name, kv.first.c_str(), sizeof(o.name) - 1);
            o.launches = kv.second.launches;
            o.ms = kv.second.ms;
            o.flops = kv.second.flops;
            o.bytes = kv.second.bytes;
        }
        ++i;
    }
    *n_out = i;
    if (ctx->prof->failed) {
        ctx->err = "gw_profile_read: some launches could not be timed";
        return GW_E_DEVICE;
    }
    return GW_OK;
}

gw_status gw_profile_end(gw_ctx *ctx) {
    if (!ctx) return GW_E_INVALID;
    if (ctx->prof) {
        if (gwk::g_prof == ctx->prof) gwk::g_prof = nullptr;
        gwk::destroy(ctx->prof);
        ctx->prof = nullptr;
    }
    return GW_OK;
}

}  // extern "C"

void gwk_prof_release(gw_ctx *c) { (void)gw_profile_end(c); }
