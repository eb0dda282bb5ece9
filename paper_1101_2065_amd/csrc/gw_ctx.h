// Private definition of the context behind the opaque gw_ctx handle.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <vector>
#include <string>

struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct GwServe;  // serving state (gw_serve.cpp)
namespace gwk {
struct ProfSink;  // kernel timing (gw_prof.cpp)
}

struct gw_ctx {
    int device = 0;
    size_t budget = 0;
    std::string err;
    bool sticky = false;
    std::map<std::string, DevBuf> bufs;
    // cached Cauchy-kernel spectrum
    int ks_n = 0;
    double ks_min = 0, ks_d = 0, ks_eps = 0;
    // set for the private contexts of serving slots: the only stream they use
    hipStream_t own_stream = nullptr;
    GwServe *serve = nullptr;
    uint64_t batch_generation = 0;
    gwk::ProfSink *prof = nullptr;
    // second stream of the FP64 solve (frequency batches on two streams) and
    // the events that fork it from and join it to the caller's stream
    hipStream_t aux = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    // one event per histogram chunk of the pipelined A route
    std::vector<hipEvent_t> chunk_ev;
};

void gwk_ctx_trim(gw_ctx *c);
size_t gwk_ctx_bytes(const gw_ctx *c);
hipError_t gwk_malloc_async(void **p, size_t bytes, hipStream_t st);
void gwk_serve_stop(gw_ctx *c);
void gwk_prof_release(gw_ctx *c);
size_t gwk_solve_ws_bytes(int n, int n_omega, bool mixed, size_t budget);
// Device address of the fixed workspace of gw_solve_W_A_noalloc on `device`
// (current), looked up once per device.
void gwk_noalloc_init(int device);
