"""The library's C ABI layer built for the host alone (no GPU): the host
sources of libgw.so (argument checks, planning, refinement driver, batch
recorder, serving loop, autotuner table, kernel timing) compiled with g++
under the address and undefined-behaviour sanitizers against a stand-in HIP
runtime (tests/hostbuild/hip/hip_runtime.h: host memory, no kernels; the
kernel launchers are stubs generated from the library's own declarations).

It exercises without a GPU what a GPU run cannot force safely: the status
codes of every argument check, the sticky device error, and the host-forced
faults of GW_FAULT (oom: workspace allocation fails; device: every checked
runtime call fails; noconv: refinement never converges, so every frequency
falls back to FP64), plus the serving queue's states, cancellation and the
one re-queue of a request that ran out of memory."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1101_2065_amd", "csrc")
STUB = os.path.join(ROOT, "tests", "hostbuild")
HOST_SOURCES = ["gw_abi.cpp", "gw_batch.cpp", "gw_serve.cpp", "gw_prof.cpp", "gw_tune.cpp", "gw_group.cpp"]


def _strip_defaults(params):
    out, depth, cur = [], 0, ""
    for ch in params:
        if ch == "(":
            depth += 1
        elif ch == ")":
            depth -= 1
        if ch == "," and depth == 0:
            out.append(cur)
            cur = ""
        else:
            cur += ch
    if cur.strip():
        out.append(cur)
    return ", ".join(p.split("=")[0].strip() for p in out)


def _launcher_stubs():
    """Definitions (returning success) of every kernel launcher the host
    sources declare in namespace gwk, from gw_internal.h and the local
    declaration blocks of the .cpp files."""
    texts = [open(os.path.join(CSRC, "gw_internal.h")).read()]
    for f in HOST_SOURCES:
        src = open(os.path.join(CSRC, f)).read()
        texts += re.findall(r"namespace gwk \{(.*?)\n\}", src, flags=re.S)
    seen, defs = set(), []
    for t in texts:
        t = re.sub(r"//[^\n]*", "", t)
        for m in re.finditer(r"(template\s*<typename Z>\s*)?(hipError_t|size_t)\s+(\w+)\s*\(([^;{]*)\)\s*;", t):
            tmpl, ret, name, params = m.group(1), m.group(2), m.group(3), m.group(4)
            params = " ".join(_strip_defaults(params).split())
            variants = [("", params)]
            if tmpl:
                variants = [("template <> ", params.replace("Z *", "%s *" % z).replace("const Z", "const %s" % z))
                            for z in ("zdbl", "zflt")]
                name_t = [name + "<zdbl>", name + "<zflt>"]
            for i, (pre, ps) in enumerate(variants):
                nm = name_t[i] if tmpl else name
                key = nm + "(" + re.sub(r"\b\w+\s*(,|$)", r"\1", ps) + ")"
                if key in seen:
                    continue
                seen.add(key)
                body = "return hipSuccess;" if ret == "hipError_t" else "return 1;"
                defs.append("%s%s %s(%s) { %s }" % (pre, ret, nm, ps, body))
    return ("// generated: every launcher succeeds without doing anything\n"
            "#include \"gw_internal.h\"\n#include \"gw_plan.h\"\n"
            "namespace gwk {\n" + "\n".join(defs) + "\n"
            "thread_local OpRecorder *g_rec = nullptr;\n"
            "int gemm_queue_occupancy(int key) { return 1 + key % 4; }\n"
            "void gemm_queue_tile(int key, int *bm, int *bn) { *bm = key % 4 == 2 ? 64 : 128; *bn = 32; }\n"
            "}  // namespace gwk\n"
            "namespace gwp {\nvoid set_thread_gemm_tile(int) {}\n"
            "bool set_thread_cgemm_bf16x(bool on) { static thread_local bool v = false; bool p = v; v = on; "
            "return p; }\n}  // namespace gwp\n"
            "void gwk_noalloc_init(int) {}\n")


DRIVER = r'''
#include "gw.h"
#include "gw_ctx.h"
#include "gw_plan.h"
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

static int fails = 0;
#define CHECK(c) do { if (!(c)) { std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); ++fails; } } while (0)

// a 2-orbital, 2-product molecule in host memory (the stand-in device memory)
struct Mol {
    std::vector<double> eig{-0.5, 0.7}, X{1, 0, 0, 1}, vals{1, 0.2, 0.2, 1, 0.5, 0, 0, 0.5}, v{1, 0.3, 0.3, 1};
    std::vector<int32_t> blk_prod{0, 2}, blk_orb{0, 2}, orb_idx{0, 1};
    std::vector<int64_t> blk_val{0, 8};
    gw_molecule m() {
        gw_molecule r{};
        r.n_orb = 2; r.n_occ = 1; r.n_prod = 2; r.eig = eig.data(); r.X = X.data(); r.n_blk = 1;
        r.blk_prod = blk_prod.data(); r.blk_orb = blk_orb.data(); r.orb_idx = orb_idx.data();
        r.blk_val = blk_val.data(); r.vals = vals.data();
        return r;
    }
};

static gw_grid grid(int n = 64) { return gw_grid{n, -2.0, 2.0, 0.1, -1}; }

int main(int argc, char **argv) {
    const std::string mode = argc > 1 ? argv[1] : "";
    gw_ctx *c = nullptr;
    CHECK(gw_create(0, 0, nullptr) == GW_E_INVALID);
    CHECK(gw_create(3, 0, &c) == GW_E_INVALID);
    CHECK(gw_create(0, 1ull << 34, &c) == GW_OK && c);
    Mol mol;
    gw_molecule m = mol.m();
    gw_grid g = grid();
    std::vector<double> chi(2 * 64 * 4), W(2 * 64 * 4);
    gw_report rep{};
    if (mode == "args") {
        CHECK(gw_build_chi0(nullptr, &m, &g, nullptr, 0, nullptr, nullptr, chi.data(), nullptr) == GW_E_INVALID);
        gw_grid bad = g; bad.n_omega = 100;
        CHECK(gw_build_chi0(c, &m, &bad, nullptr, 0, nullptr, nullptr, chi.data(), nullptr) == GW_E_INVALID);
        CHECK(std::strstr(gw_last_error(c), "power of two"));
        bad = g; bad.omega_max = 3.0;
        CHECK(gw_build_chi0(c, &m, &bad, nullptr, 0, nullptr, nullptr, chi.data(), nullptr) == GW_E_INVALID);
        bad = g; bad.eps = 0.0;
        CHECK(gw_build_chi0(c, &m, &bad, nullptr, 0, nullptr, nullptr, chi.data(), nullptr) == GW_E_INVALID);
        Mol m2; m2.eig = {0.7, -0.5};
        gw_molecule mm = m2.m();
        CHECK(gw_build_chi0(c, &mm, &g, nullptr, 0, nullptr, nullptr, chi.data(), nullptr) == GW_E_INVALID);
        CHECK(std::strstr(gw_last_error(c), "ascending"));
        Mol m3; m3.orb_idx = {0, 5};
        mm = m3.m();
        CHECK(gw_build_chi0(c, &mm, &g, nullptr, 0, nullptr, nullptr, chi.data(), nullptr) == GW_E_INVALID);
        CHECK(std::strstr(gw_last_error(c), "out of range"));
        Mol m4; m4.blk_val = {0, 7};
        mm = m4.m();
        CHECK(gw_build_chi0(c, &mm, &g, nullptr, 0, nullptr, nullptr, chi.data(), nullptr) == GW_E_INVALID);
        CHECK(gw_build_chi0(c, &m, &g, nullptr, 0, nullptr, nullptr, nullptr, nullptr) == GW_E_INVALID);
        CHECK(gw_solve_W(c, mol.v.data(), 0, 2, chi.data(), 63, GW_FP64, 1e-7, nullptr, W.data(), nullptr) == GW_E_INVALID);
        CHECK(gw_solve_W(c, mol.v.data(), 0, 0, chi.data(), 64, GW_FP64, 1e-7, nullptr, W.data(), nullptr) == GW_E_INVALID);
        CHECK(gw_solve_W(c, mol.v.data(), 0, 2, chi.data(), 64, (gw_precision)7, 1e-7, nullptr, W.data(), nullptr) == GW_E_INVALID);
        CHECK(gw_solve_W(c, mol.v.data(), 0, 2, chi.data(), 64, GW_FP32_IR, 0.0, nullptr, W.data(), nullptr) == GW_E_INVALID);
        setenv("GW_A_TRANSFORM", "fft", 1);  // the FFT form takes 128 to 1024 points only
        CHECK(gw_build_A(c, &m, mol.v.data(), &g, nullptr, chi.data(), nullptr) == GW_E_INVALID);
        unsetenv("GW_A_TRANSFORM");
        CHECK(gw_build_A(c, &m, mol.v.data(), &g, nullptr, chi.data(), nullptr) == GW_OK);
        CHECK(gw_build_A_compressed(c, &m, mol.v.data(), nullptr, 2, &g, nullptr, chi.data(), nullptr) == GW_E_INVALID);
        CHECK(gw_compress_basis(c, mol.v.data(), 2, 3, nullptr, W.data(), W.data()) == GW_E_INVALID);
        CHECK(gw_decompress(c, mol.v.data(), 2, 0, chi.data(), nullptr, nullptr, W.data()) == GW_E_INVALID);
        // valid calls run through planning and the (stub) launches
        CHECK(gw_build_chi0(c, &m, &g, nullptr, 0, nullptr, nullptr, chi.data(), &rep) == GW_OK);
        CHECK(rep.n_hbins >= 2);
        CHECK(gw_solve_W(c, mol.v.data(), 0, 2, chi.data(), 64, GW_FP64, 1e-7, nullptr, W.data(), &rep) == GW_OK);
        CHECK(rep.n_solved == 33 && rep.n_fallback == 0);
        CHECK(gw_solve_W(c, mol.v.data(), 0, 2, chi.data(), 64, GW_BF16X_IR, 1e-7, nullptr, W.data(), &rep) == GW_OK);
        CHECK(rep.n_fallback == 0);
        // batch: create, run, retire by a newer batch
        const double *vs[1] = {mol.v.data()};
        void *cs[1] = {chi.data()}, *ws[1] = {W.data()};
        gw_batch *b = nullptr, *b2 = nullptr;
        CHECK(gw_batch_create(c, 1, &m, vs, &g, GW_FP64, 1e-7, 0, nullptr, cs, ws, &b) == GW_OK);
        CHECK(gw_batch_run(b, nullptr, &rep) == GW_OK);
        CHECK(gw_batch_create(c, 1, &m, vs, &g, GW_FP64, 1e-7, 0, nullptr, cs, ws, &b2) == GW_OK);
        CHECK(gw_batch_run(b, nullptr, &rep) == GW_E_STATE);
        CHECK(gw_batch_run(b2, nullptr, &rep) == GW_OK);
        CHECK(gw_batch_destroy(b) == GW_OK);
        gw_batch *b3 = nullptr;
        CHECK(gw_batch_create(c, 1, &m, vs, &g, GW_FP32_IR, 1e-7, 0, nullptr, cs, ws, &b3) == GW_E_INVALID);
        CHECK(b3 == nullptr);
        CHECK(gw_batch_destroy(b2) == GW_OK);
    } else if (mode == "oom") {
        CHECK(gw_build_chi0(c, &m, &g, nullptr, 0, nullptr, nullptr, chi.data(), nullptr) == GW_E_OOM);
        CHECK(std::strstr(gw_last_error(c), "GW_FAULT=oom"));
        CHECK(gw_solve_W(c, mol.v.data(), 0, 2, chi.data(), 64, GW_FP64, 1e-7, nullptr, W.data(), nullptr) == GW_E_OOM);
        // not sticky: the context stays usable
        CHECK(gw_build_chi0(c, &m, &g, nullptr, 0, nullptr, nullptr, chi.data(), nullptr) == GW_E_OOM);
    } else if (mode == "device") {
        CHECK(gw_build_chi0(c, &m, &g, nullptr, 0, nullptr, nullptr, chi.data(), nullptr) == GW_E_DEVICE);
        CHECK(gw_solve_W(c, mol.v.data(), 0, 2, chi.data(), 64, GW_FP64, 1e-7, nullptr, W.data(), nullptr) == GW_E_DEVICE);
        CHECK(std::strstr(gw_last_error(c), "sticky"));
        uint64_t t = 0;
        CHECK(gw_submit(c, &m, mol.v.data(), &g, 0, GW_FP64, 1e-7, &t) == GW_E_DEVICE);
    } else if (mode == "noconv") {
        CHECK(gw_solve_W(c, mol.v.data(), 0, 2, chi.data(), 64, GW_FP32_IR, 1e-7, nullptr, W.data(), &rep) == GW_OK);
        CHECK(rep.n_solved == 33 && rep.n_fallback == 33);
        CHECK(gw_solve_W(c, mol.v.data(), 0, 2, chi.data(), 64, GW_FP64, 1e-7, nullptr, W.data(), &rep) == GW_OK);
        CHECK(rep.n_fallback == 0);
        const double *vs[1] = {mol.v.data()};
        void *cs[1] = {chi.data()}, *ws[1] = {chi.data()};  // in place: no FP64 re-solve possible
        gw_batch *b = nullptr;
        CHECK(gw_batch_create(c, 1, &m, vs, &g, GW_BF16X_IR, 1e-7, 2, nullptr, cs, ws, &b) == GW_OK);
        CHECK(gw_batch_run(b, nullptr, &rep) == GW_E_NOCONV);
        gw_batch_destroy(b);
    } else if (mode == "serve" || mode == "serve_oom") {
        const bool oom = mode == "serve_oom";
        uint64_t t[3];
        for (int i = 0; i < 3; ++i) CHECK(gw_submit(c, &m, mol.v.data(), &g, 0, GW_FP64, 1e-7, &t[i]) == GW_OK);
        CHECK(gw_poll(c, 999, nullptr, nullptr) == GW_E_STATE);
        CHECK(gw_release(c, 999) == GW_E_STATE);
        int left = 3, spins = 0;
        bool done[3] = {false, false, false};
        while (left && spins++ < 200000) {
            for (int i = 0; i < 3; ++i) {
                if (done[i]) continue;
                void *p = nullptr;
                gw_status s = gw_poll(c, t[i], &p, &rep);
                if (s == GW_PENDING) continue;
                if (oom) {
                    CHECK(s == GW_E_OOM);
                    CHECK(std::strstr(gw_last_error(c), "after one retry"));
                } else {
                    CHECK(s == GW_OK && p != nullptr && rep.n_solved == 33);
                }
                CHECK(gw_release(c, t[i]) == GW_OK);
                CHECK(gw_poll(c, t[i], nullptr, nullptr) == GW_E_STATE);
                done[i] = true;
                --left;
            }
        }
        CHECK(left == 0);
        gw_molecule bad = m; bad.n_occ = 2;
        uint64_t tb;
        CHECK(gw_submit(c, &bad, mol.v.data(), &g, 0, GW_FP64, 1e-7, &tb) == GW_E_INVALID);
        CHECK(gw_submit(c, &m, mol.v.data(), &g, 3, GW_FP64, 1e-7, &tb) == GW_E_INVALID);
    } else if (mode == "hist_ranges") {
        // the A route's bin ranges: pair bins [0, nhb - 1) and product bins
        // [1, nhb) each covered once and in order, products of at most dchunk
        // bins, every product bin final when its range is done
        std::vector<gwp::HistRange> rg;
        for (int nhb = 0; nhb <= 300; ++nhb)
            for (int dchunk : {1, 2, 3, 5, 67, 1000})
                for (int want : {1, 2, 3, 4, 7, 64}) {
                    gwp::hist_ranges(nhb, dchunk, want, &rg);
                    if (nhb <= 1) {
                        CHECK(rg.empty());
                        continue;
                    }
                    int next_lo = 0, next_m = 1;
                    for (const gwp::HistRange &r : rg) {
                        CHECK(r.lo == next_lo && r.hi >= r.lo && r.hi <= nhb - 1);
                        CHECK(r.m0 == next_m && r.cnt >= 1 && r.cnt <= dchunk);
                        CHECK(r.hi >= std::min(r.m0 + r.cnt, nhb - 1));
                        next_lo = r.hi;
                        next_m = r.m0 + r.cnt;
                    }
                    CHECK(next_lo == nhb - 1 && next_m == nhb);
                    CHECK((int)rg.size() <= std::max(want, (nhb - 1 + dchunk - 1) / dchunk));
                }
    } else if (mode == "lockstep") {
        // two recorded programs: products, a panel, its row exchanges and a
        // deferred launch, against two products of a second molecule
        int ran = 0;
        auto gemm = [](int M, int N, int K, int batch) {
            gwk::RecOp o;
            o.kind = gwk::RecOp::GEMM;
            o.key = gwk::QK_Z3M * 4 + 2;
            o.g.M = M; o.g.N = N; o.g.K = K; o.g.batch = batch;
            o.flops = 8.0 * M * N * K * batch;
            return o;
        };
        gwk::RecOp pan, swp, oth, mark;
        pan.kind = gwk::RecOp::PANEL; pan.key = 1;
        pan.p.n = 300; pan.p.w = 64; pan.p.kb = 0; pan.p.batch = 5;
        swp = pan; swp.kind = gwk::RecOp::LASWP; swp.key = 0;
        oth.kind = gwk::RecOp::OTHER;
        oth.fn = [&ran](hipStream_t) { ++ran; return hipSuccess; };
        mark.kind = gwk::RecOp::MARK;
        for (int align = 0; align < 2; ++align) {
            std::vector<std::vector<gwk::RecOp>> progs(2);
            progs[0] = {mark, gemm(100, 70, 64, 3), pan, swp, oth, mark};
            progs[1] = {gemm(40, 40, 16, 2), mark, gemm(100, 70, 64, 1)};
            gwp::LockStep *ls = nullptr;
            CHECK(gwp::lockstep_plan(c, progs, align == 1, &ls) == GW_OK && ls);
            const gwp::LockStepStats st = gwp::lockstep_stats(ls);
            CHECK(st.steps == 4 && st.ops == 6 && st.products == 3);
            // right-aligned: {G0} {P0} {S0, G1} {O0, G1}; left: {G0 G1} {P0, G1} {S0} {O0}
            CHECK(st.launches == (align ? 6 : 5));
            const gwk::GemmItem *gi = (const gwk::GemmItem *)c->bufs["lsGemm"].ptr;
            const gwk::PanelItem *pi = (const gwk::PanelItem *)c->bufs["lsPanel"].ptr;
            // 64 x 32 tiles: 100 x 70 in 2 x 3, times the batch
            CHECK(gi[0].M == 100 && gi[0].tx == 3 && gi[0].ty == 2 && gi[0].t0 == 0);
            if (align) {
                CHECK(gi[1].M == 40 && gi[1].t0 == 0 && gi[1].tx == 2 && gi[1].ty == 1);
                CHECK(gi[2].M == 100 && gi[2].batch == 1 && gi[2].t0 == 0);
            } else {
                CHECK(gi[1].M == 40 && gi[1].t0 == 18);  // after the first item's 2 x 3 x 3 tiles
                CHECK(gi[2].M == 100 && gi[2].batch == 1 && gi[2].t0 == 0);
            }
            CHECK(pi[0].batch == 5 && pi[0].wg0 == 0 && pi[1].wg0 == 0 && pi[1].n == 300);
            std::vector<hipStream_t> br(2);
            std::vector<hipEvent_t> ev(3);
            for (auto &x : br) hipStreamCreateWithFlags(&x, 0);
            for (auto &x : ev) hipEventCreate(&x);
            CHECK(gwp::lockstep_enqueue(c, *ls, nullptr, br, ev) == GW_OK);
            CHECK(ran == align + 1);
            CHECK(gwp::lockstep_enqueue(c, *ls, nullptr, br, {}) == GW_E_INVALID);
            gwp::lockstep_free(ls);
        }
        int32_t md = -1;
        int64_t nst = -1;
        const double *vs[1] = {mol.v.data()};
        void *cs[1] = {chi.data()}, *ws[1] = {W.data()};
        gw_batch *b = nullptr;
        CHECK(gw_batch_stats(nullptr, &md, &nst, nullptr, nullptr) == GW_E_INVALID);
        CHECK(gw_batch_create(c, 1, &m, vs, &g, GW_FP64, 1e-7, 0, nullptr, cs, ws, &b) == GW_OK);
        CHECK(gw_batch_stats(b, &md, &nst, nullptr, nullptr) == GW_OK && md == 1 && nst == 0);
        CHECK(gw_batch_run(b, nullptr, &rep) == GW_OK);
        CHECK(gw_batch_destroy(b) == GW_OK);
    } else {
        std::printf("unknown mode\n");
        return 2;
    }
    CHECK(gw_destroy(c) == GW_OK);
    std::printf(fails ? "FAILED %d\n" : "OK\n", fails);
    std::fflush(stdout);
    return fails ? 1 : 0;
}
'''


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("hostbuild")
    (d / "stubs.cpp").write_text(_launcher_stubs())
    (d / "driver.cpp").write_text(DRIVER)
    exe = d / "driver"
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-pthread", "-I", STUB, "-I", CSRC, "-I", os.path.join(ROOT, "include")]
    srcs = [os.path.join(CSRC, f) for f in HOST_SOURCES] + [str(d / "stubs.cpp"), str(d / "driver.cpp")]
    r = subprocess.run(["g++"] + flags + srcs + ["-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return str(exe), str(d)


def _run(drv, mode, fault=None, extra_env=None):
    exe, d = drv
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1",
               GW_TUNE_FILE=os.path.join(d, "tune.json"))
    env.pop("GW_FAULT", None)
    env.pop("GW_SERVE_CHI0", None)
    if fault:
        env["GW_FAULT"] = fault
    env.update(extra_env or {})
    r = subprocess.run([exe, mode], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout[-3000:] + r.stderr[-3000:]


def test_argument_checks_and_status_codes(driver):
    _run(driver, "args")


@pytest.mark.parametrize("fault", ["oom", "device", "noconv"])
def test_forced_faults(driver, fault):
    _run(driver, fault, fault)


def test_lock_step_grouping(driver):
    """The batched driver's lock steps: operation k of every recorded program
    in step k (or aligned at the end), the products of a step in one
    work-queue launch with consecutive tile ranges, panels and row exchanges
    grouped with their workgroup offsets, deferred launches run once."""
    _run(driver, "lockstep")


def test_a_route_histogram_ranges(driver):
    """The A route's histogram ranges and product chunks over 301 bin counts,
    six staging sizes and six range counts: each bin once, in order, final
    before its product."""
    _run(driver, "hist_ranges")


@pytest.mark.parametrize("route", ["A", "chi0"])
def test_serving_states(driver, route):
    """Served requests form A in W's buffer and solve in place, or with
    GW_SERVE_CHI0=1 form chi0 in a buffer of their own first."""
    _run(driver, "serve", extra_env={"GW_SERVE_CHI0": "1"} if route == "chi0" else None)


def test_serving_requeues_once_after_running_out_of_memory(driver):
    _run(driver, "serve_oom", "oom")
