// Schedule cache of fit_plan_tune (host code only; no HIP): a text file, one
// line per tuned shape, "<key>\t<waves> <waves_per_block> <tile> <unroll> <ms>"
// and, optionally, " <graph>": 1 when replaying a captured graph was the
// faster form, 0 when eager launches were (a line without it leaves the form
// to the plan).
// The key names the device (architecture and compute units) and the shape of
// the call (dtype, options, batch, and the total points rounded down to a
// power of two); the last line with a key wins.  Lines that do not parse are
// skipped; a file that cannot be read is treated as empty and one that cannot
// be written is left alone.  Lookups and appends within a process are
// serialised by one mutex.
#pragma once

#include <cstdint>
#include <cstdio>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>

#include "lsefit.h"

namespace lsefit {
namespace tune_cache {

inline std::mutex& file_mutex() {
    static std::mutex mu;
    return mu;
}

inline std::string key(const std::string& arch, int cus, const lsefit_options* opt, int32_t dt, int64_t batch,
                       int64_t points) {
    int lg = 0;
    while (lg < 62 && (int64_t(1) << (lg + 1)) <= points) ++lg;
    char buf[320];
    std::snprintf(buf, sizeof buf, "%.64s cu=%d dt=%d prec=%d refine=%d basis=%d solver=%d range=%d m=%d B=%lld N=2^%d",
                  arch.c_str(), cus, dt, opt->precision, opt->refine_steps, opt->basis, opt->solver,
                  opt->range_mode, opt->degree, (long long)batch, lg);
    return buf;
}

// the schedule and time of the last parsable line for `key`, if any, and its
// replay form in *graph (0 or 1; -1 when the line does not give one)
inline bool lookup(const std::string& path, const std::string& key, lsefit_schedule* s, double* ms,
                   int* graph = nullptr) {
    std::lock_guard<std::mutex> g(file_mutex());
    std::ifstream in(path);
    if (!in) return false;
    bool found = false;
    std::string line;
    while (std::getline(in, line)) {
        const size_t tab = line.find('\t');
        if (tab == std::string::npos || tab != key.size() || line.compare(0, tab, key) != 0) continue;
        std::istringstream vals(line.substr(tab + 1));
        lsefit_schedule c{};
        double t = 0.0;
        if (vals >> c.waves >> c.waves_per_block >> c.tile >> c.unroll >> t) {
            int gr = -1;
            if (!(vals >> gr) || (gr != 0 && gr != 1)) gr = -1;
            *s = c;
            *ms = t;
            if (graph) *graph = gr;
            found = true;
        }
    }
    return found;
}

// appends one line (with the replay form when graph is 0 or 1); a last line
// left without its newline (an interrupted write) is ended first, so that the
// new line stands on its own
inline void store(const std::string& path, const std::string& key, const lsefit_schedule& s, double ms,
                  int graph = -1) {
    std::lock_guard<std::mutex> g(file_mutex());
    FILE* f = std::fopen(path.c_str(), "a+");
    if (!f) return;
    const bool ended = std::fseek(f, -1, SEEK_END) != 0 || std::fgetc(f) == '\n';   // empty, or ends a line
    std::fseek(f, 0, SEEK_END);   // a read is followed by a write only after a positioning call
    if (!ended) std::fputc('\n', f);
    std::fprintf(f, "%s\t%d %d %d %d %.6f", key.c_str(), s.waves, s.waves_per_block, s.tile, s.unroll, ms);
    if (graph == 0 || graph == 1) std::fprintf(f, " %d", graph);
    std::fputc('\n', f);
    std::fclose(f);
}

}  // namespace tune_cache
}  // namespace lsefit
