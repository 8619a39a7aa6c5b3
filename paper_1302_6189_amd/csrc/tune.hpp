// tune.hpp -- parameters chosen by the autotuner (autotune.hip) and applied
// by plans built for the batched form.
#pragma once

#include <map>
#include <string>
#include <utility>
#include <vector>

namespace fftrw {

struct RowTune {
    int rows_per_wg = 0;      // 0: built-in choice
    std::vector<int> radix;   // empty: built-in factorisation
};

struct TileTune {
    int TU = 0, TV = 0, G = 0;  // 0: built-in choice
};

struct TuneTable {
    std::string device, version;
    std::map<int, RowTune> rows;                       // by row length
    std::map<std::pair<int, int>, TileTune> tiles;     // by (Nu, Nv)
    std::map<std::pair<int, int>, std::vector<int>> fused;  // radix order of a fused step, by (N, Nv)
};

// Load a cache written by fft_autotune; false if missing, unreadable, or
// made for another device or library version.
bool tune_load(const std::string &path, const std::string &device, const std::string &version, TuneTable *out);
bool tune_save(const std::string &path, const TuneTable &t);
std::string tune_device_name();

}  // namespace fftrw
