// Autotuner table file (see gw_tune.h).  Plain C++ and POSIX calls only.
#include "gw_tune.h"

#include <errno.h>
#include <stdio.h>
#include <sys/stat.h>
#include <sys/types.h>
#include <unistd.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

namespace gwt {

std::string cache_path() {
    if (const char *e = std::getenv("GW_TUNE_FILE")) return e;
    const char *h = std::getenv("HOME");
    return std::string(h ? h : "/tmp") + "/.cache/gw_tune.json";
}

bool load(const std::string &path, std::map<std::string, int> *table, std::string *err) {
    std::ifstream f(path);
    if (!f) {
        struct stat sb;
        if (::stat(path.c_str(), &sb) != 0 && errno == ENOENT) return true;  // no table yet
        *err = "cannot read " + path;
        return false;
    }
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    std::map<std::string, int> got;
    size_t p = t.find('{');
    if (p == std::string::npos) {
        *err = path + ": not a JSON object";
        return false;
    }
    // {"key": integer, ...}: keys are written by save() and hold no quotes
    while (true) {
        p = t.find_first_of("\"}", p + 1);
        if (p == std::string::npos) {
            *err = path + ": unterminated object";
            return false;
        }
        if (t[p] == '}') break;
        const size_t q = t.find('"', p + 1);
        if (q == std::string::npos) {
            *err = path + ": unterminated key";
            return false;
        }
        const std::string key = t.substr(p + 1, q - p - 1);
        const size_t c = t.find(':', q);
        if (c == std::string::npos) {
            *err = path + ": missing ':' after key " + key;
            return false;
        }
        char *end = nullptr;
        const long v = std::strtol(t.c_str() + c + 1, &end, 10);
        if (end == t.c_str() + c + 1) {
            *err = path + ": value of " + key + " is not an integer";
            return false;
        }
        got[key] = (int)v;
        p = (size_t)(end - t.c_str());
        const size_t nx = t.find_first_of(",}", p);
        if (nx == std::string::npos) {
            *err = path + ": unterminated object";
            return false;
        }
        if (t[nx] == '}') break;
        p = nx;
    }
    for (auto &kv : got) (*table)[kv.first] = kv.second;
    return true;
}

bool make_dirs(const std::string &dir, std::string *err) {
    if (dir.empty()) return true;
    std::string cur;
    size_t i = 0;
    if (dir[0] == '/') {
        cur = "/";
        i = 1;
    }
    while (i <= dir.size()) {
        size_t j = dir.find('/', i);
        if (j == std::string::npos) j = dir.size();
        if (j > i) {
            cur += dir.substr(i, j - i);
            if (::mkdir(cur.c_str(), 0755) != 0 && errno != EEXIST) {
                *err = "cannot create directory " + cur + ": " + std::strerror(errno);
                return false;
            }
            struct stat sb;
            if (::stat(cur.c_str(), &sb) != 0 || !S_ISDIR(sb.st_mode)) {
                *err = cur + " exists and is not a directory";
                return false;
            }
            cur += '/';
        }
        i = j + 1;
    }
    return true;
}

bool save(const std::string &path, const std::map<std::string, int> &table, std::string *err) {
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0 && !make_dirs(path.substr(0, slash), err)) return false;
    const std::string tmp = path + ".tmp" + std::to_string((long)::getpid());
    {
        std::ofstream f(tmp);
        if (!f) {
            *err = "cannot write " + tmp;
            return false;
        }
        f << "{";
        bool first = true;
        for (auto &kv : table) {
            f << (first ? "" : ", ") << "\"" << kv.first << "\": " << kv.second;
            first = false;
        }
        f << "}\n";
        f.flush();
        if (!f) {
            *err = "write to " + tmp + " failed";
            (void)::unlink(tmp.c_str());
            return false;
        }
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) {
        *err = "cannot rename " + tmp + " to " + path + ": " + std::strerror(errno);
        (void)::unlink(tmp.c_str());
        return false;
    }
    return true;
}

double median(std::vector<double> v) {
    std::sort(v.begin(), v.end());
    const size_t n = v.size();
    return n % 2 ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]);
}

}  // namespace gwt
