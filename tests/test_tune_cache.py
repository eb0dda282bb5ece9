"""The autotuner's table file, built for the host alone with g++ under the
address and undefined-behaviour sanitizers (no GPU needed): directories are
made with mkdir(2), so a path holding quotes, spaces or shell syntax is only a
path; the table round-trips; failures are reported, not swallowed."""
import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1101_2065_amd", "csrc")

DRIVER = r'''
#include "gw_tune.h"
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
// usage: driver save PATH | load PATH | median
int main(int argc, char **argv) {
    if (argc >= 2 && !std::strcmp(argv[1], "median")) {
        std::printf("%g %g\n", gwt::median({3, 1, 2}), gwt::median({4, 1, 3, 2}));
        return 0;
    }
    if (argc < 3) return 2;
    std::string err;
    std::map<std::string, int> t;
    if (!std::strcmp(argv[1], "save")) {
        t["zgemm_fp64_n2048"] = 3;
        t["cgemm_fp32_n512"] = 1;
        if (!gwt::save(argv[2], t, &err)) { std::printf("ERR %s\n", err.c_str()); return 1; }
        std::printf("OK\n");
        return 0;
    }
    if (!std::strcmp(argv[1], "load")) {
        t["kept"] = 7;
        if (!gwt::load(argv[2], &t, &err)) { std::printf("ERR %s\n", err.c_str()); return 1; }
        for (auto &kv : t) std::printf("%s=%d\n", kv.first.c_str(), kv.second);
        return 0;
    }
    return 2;
}
'''


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("tune")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, str(src), os.path.join(CSRC, "gw_tune.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return str(exe)


def _run(exe, *args, cwd=None):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([exe, *args], capture_output=True, text=True, cwd=cwd, env=env)


def test_save_under_a_path_with_quotes_and_shell_syntax(driver, tmp_path):
    base = tmp_path / "it's here" / "$(touch INJECTED)" / "a b"
    path = base / "tune.json"
    r = _run(driver, "save", str(path), cwd=str(tmp_path))
    assert r.returncode == 0 and r.stdout.strip() == "OK", r.stdout + r.stderr
    assert json.loads(path.read_text()) == {"cgemm_fp32_n512": 1, "zgemm_fp64_n2048": 3}
    assert not (tmp_path / "INJECTED").exists()
    assert [p.name for p in base.iterdir()] == ["tune.json"]  # no temporary left behind
    r = _run(driver, "load", str(path))
    assert r.returncode == 0, r.stderr
    assert r.stdout.split() == ["cgemm_fp32_n512=1", "kept=7", "zgemm_fp64_n2048=3"]


def test_missing_table_is_empty_and_bad_tables_are_reported(driver, tmp_path):
    r = _run(driver, "load", str(tmp_path / "absent.json"))
    assert r.returncode == 0 and r.stdout.split() == ["kept=7"]
    bad = tmp_path / "bad.json"
    bad.write_text('{"zgemm_fp64_n256": }')
    r = _run(driver, "load", str(bad))
    assert r.returncode == 1 and r.stdout.startswith("ERR")
    bad.write_text('{"zgemm_fp64_n256": 2')
    r = _run(driver, "load", str(bad))
    assert r.returncode == 1 and "unterminated" in r.stdout


def test_unwritable_path_is_reported(driver, tmp_path):
    blocker = tmp_path / "file"
    blocker.write_text("x")
    r = _run(driver, "save", str(blocker / "sub" / "tune.json"))
    assert r.returncode == 1 and r.stdout.startswith("ERR") and "not a directory" in r.stdout


def test_median(driver):
    r = _run(driver, "median")
    assert r.returncode == 0 and r.stdout.split() == ["2", "2.5"]
