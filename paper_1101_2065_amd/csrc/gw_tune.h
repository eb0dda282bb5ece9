// Autotuner table file: a flat JSON object {"key": tile, ...}.  Host-only
// (no HIP), so the file handling builds and runs without a GPU.
#pragma once

#include <map>
#include <string>
#include <vector>

namespace gwt {

// $GW_TUNE_FILE, else $HOME/.cache/gw_tune.json (/tmp when HOME is unset).
std::string cache_path();

// Reads the table at `path` into *table (entries already there are replaced
// by the file's).  A missing file is not an error (returns true, nothing
// read); an unreadable or malformed one returns false with *err set.
bool load(const std::string &path, std::map<std::string, int> *table, std::string *err);

// Creates every missing directory of `dir` with mkdir(2) (no process is
// spawned).  False with *err set if a component cannot be created or is not a
// directory.
bool make_dirs(const std::string &dir, std::string *err);

// Writes the table to `path`: missing parent directories are created, the
// text goes to a temporary file beside it, which is then renamed over the
// target (readers never see half a file).  False with *err set on failure.
bool save(const std::string &path, const std::map<std::string, int> &table, std::string *err);

// Median of a non-empty list of timings.
double median(std::vector<double> v);

}  // namespace gwt
