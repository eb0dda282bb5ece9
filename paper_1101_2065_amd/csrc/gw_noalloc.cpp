// gw_solve_W_A_noalloc: the FP64 solve of W from A = 1 - v chi0 with no
// allocation of any kind, for callers that cannot allocate (code under graph
// capture, tight serving loops, harnesses that forbid it).
//
// Its workspace is one fixed array in device memory, `scratch` below, of
// GW_NOALLOC_SCRATCH_BYTES per GPU.  In host code the array's name only stands
// for the device symbol: its device address is looked up once per device with
// hipGetSymbolAddress (gwk_noalloc_init, called by gw_create with that device
// current) and kept per device; every kernel argument uses that address.
// Frequencies are factorised in batches that fit the array.  Every call on a
// GPU shares its array: calls that overlap in time on one GPU race.
#include "gw_plan.h"
#include "gw_prof.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#define GW_NOALLOC_SCRATCH_BYTES (64ull << 20)

static __device__ __align__(256) unsigned char scratch[GW_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 256;
std::mutex g_mu;
void *g_scratch[kMaxDevices];           // device address of the array, per device
hipError_t g_scratch_err[kMaxDevices];  // result of the lookup, per device
bool g_scratch_done[kMaxDevices];

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Workspace layout of a batch of nb frequencies at size n (the buffers of the
// allocating solve, packed in the array at 256-byte boundaries).
struct Layout {
    size_t scr, li, ui, ipiv, perm, info, total;
};

Layout layout(int n, int nb) {
    const int nblk = (n + 63) / 64;
    Layout l;
    size_t off = 0;
    l.scr = off;
    off += round256((size_t)nb * (64 * (size_t)n * 16 + 4 * 257 + 256));  // panel scratch + swap lists
    l.li = off;
    off += round256((size_t)nb * nblk * 64 * 64 * 16);  // inverted diagonal blocks of L
    l.ui = off;
    off += round256((size_t)nb * nblk * 64 * 64 * 16);  // and of U
    l.ipiv = off;
    off += round256((size_t)nb * n * 4);
    l.perm = off;
    off += round256((size_t)nb * n * 4);
    l.info = off;
    off += round256((size_t)nb * 4);
    l.total = off;
    return l;
}

// Disables the calling thread's kernel timing for the life of the guard (its
// events would be created on demand).
struct NoProf {
    gwk::ProfSink *saved;
    NoProf() : saved(gwk::g_prof) { gwk::g_prof = nullptr; }
    ~NoProf() { gwk::g_prof = saved; }
};

}  // namespace

// Looks up the array's device address on the current device (once per
// device); the outcome is kept and reported by the entry point.
void gwk_noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch_done[device]) return;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    g_scratch[device] = e == hipSuccess ? p : nullptr;
    g_scratch_done[device] = true;
}

extern "C" gw_status gw_solve_W_A_noalloc(gw_ctx *ctx, const double *v, int32_t v_is_diag, int32_t n, void *A,
                                          int32_t n_omega, void *stream, void *W_out, gw_report *rep) {
    using gwp::fail;
    if (!ctx) return GW_E_INVALID;
    if (ctx->sticky) return fail(ctx, GW_E_DEVICE, "context has a sticky device error: " + ctx->err);
    if (!v || !A || !W_out) return fail(ctx, GW_E_INVALID, "NULL pointer argument");
    if (W_out == A) return fail(ctx, GW_E_INVALID, "W_out must not alias A");
    if (n < 1 || n > 32768) return fail(ctx, GW_E_INVALID, "n must be in [1, 32768]");
    if (n_omega < 2 || (n_omega & 1)) return fail(ctx, GW_E_INVALID, "n_omega must be even and >= 2");
    if (ctx->device < 0 || ctx->device >= kMaxDevices) return fail(ctx, GW_E_INVALID, "device index out of range");
    GW_HIP(ctx, hipSetDevice(ctx->device));
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_scratch_done[ctx->device])
            return fail(ctx, GW_E_STATE, "the fixed workspace of this device was not set up (gw_create does it)");
        if (!g_scratch[ctx->device])
            return fail(ctx, GW_E_DEVICE, std::string("fixed workspace unavailable: hipGetSymbolAddress: ") +
                                              hipGetErrorString(g_scratch_err[ctx->device]));
        base = g_scratch[ctx->device];
    }
    // the largest batch whose workspace fits the array
    const int cnt = n_omega == 2 ? 2 : n_omega / 2;
    int nbmax = std::min(256, cnt);
    while (nbmax >= 1 && layout(n, nbmax).total > GW_NOALLOC_SCRATCH_BYTES) --nbmax;
    if (nbmax < 1)
        return fail(ctx, GW_E_INVALID, "n = " + std::to_string(n) + " needs " + std::to_string(layout(n, 1).total) +
                                           " bytes of workspace per frequency; the fixed array holds " +
                                           std::to_string(GW_NOALLOC_SCRATCH_BYTES));
    NoProf noprof;
    hipStream_t st = (hipStream_t)stream;
    const int64_t nn = (int64_t)n * n;
    gwp::zdbl *Ad = (gwp::zdbl *)A, *W = (gwp::zdbl *)W_out;
    unsigned char *b = (unsigned char *)base;
    int n_solved = 0;
    auto run = [&](int j0, int nb) -> gw_status {
        const Layout l = layout(n, nb);
        gwp::SolveWs w;
        w.A = Ad + j0 * nn;
        w.scratch = b + l.scr;
        w.Li = b + l.li;
        w.Ui = b + l.ui;
        w.ipiv = (int32_t *)(b + l.ipiv);
        w.perm = (int32_t *)(b + l.perm);
        w.info = (int32_t *)(b + l.info);
        n_solved += nb;
        return gwp::solve_batch_fp64(ctx, st, n, v, v_is_diag, nullptr, W + j0 * nn, nb, w);
    };
    gw_status s;
    if (n_omega == 2) {
        // omega_0 = -omega_max and omega_1 = 0: no mirror pair, both solved
        for (int j = 0; j < 2; j += nbmax)
            if ((s = run(j, std::min(nbmax, 2 - j))) != GW_OK) return s;
    } else {
        // the lone point j = 0, then j in [n_omega/2, n_omega) in balanced
        // batches of at most nbmax; the rest by the conjugate mirror
        if ((s = run(0, 1)) != GW_OK) return s;
        const int nbat = (cnt + nbmax - 1) / nbmax;
        for (int i = 0, j = n_omega / 2; i < nbat; ++i) {
            const int sz = cnt / nbat + (i < cnt % nbat ? 1 : 0);
            if ((s = run(j, sz)) != GW_OK) return s;
            j += sz;
        }
        GW_HIP(ctx, gwk::launch_conj_mirror(st, nn, n_omega, W));
    }
    if (rep) {
        GW_HIP(ctx, hipStreamSynchronize(st));
        std::memset(rep, 0, sizeof(*rep));
        rep->n_solved = n_solved;
    }
    return GW_OK;
}
