// Host-only check of the schedule-cache file of fit_plan_tune (tune_cache.hpp),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitized.py.  Exit status 0 when every check holds.
#include <cstdio>
#include <cstdlib>
#include <string>

#include "tune_cache.hpp"

static int failures = 0;
#define CHECK(cond)                                                          \
    do {                                                                     \
        if (!(cond)) {                                                       \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            ++failures;                                                      \
        }                                                                    \
    } while (0)

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    const std::string path = std::string(argv[1]) + "/cache.txt";
    using namespace lsefit;
    lsefit_options o{};
    o.degree = 3;
    o.range_mode = 1;
    const std::string ka = tune_cache::key("gfx950", 256, &o, 0, 65536, 515205176);
    o.degree = 2;
    const std::string kb = tune_cache::key("gfx950", 256, &o, 0, 4096, 1 << 24);
    CHECK(ka != kb);
    CHECK(ka.find("N=2^28") != std::string::npos);   // 515,205,176 rounds down to 2^28
    CHECK(kb.find("N=2^24") != std::string::npos);
    CHECK(tune_cache::key("gfx950", 256, &o, 0, 1, 0).find("N=2^0") != std::string::npos);
    CHECK(tune_cache::key("gfx950", 256, &o, 0, 1, INT64_MAX).find("N=2^62") != std::string::npos);
    // an architecture name longer than the key buffer is cut, not overrun
    CHECK(tune_cache::key(std::string(4000, 'x'), 256, &o, 0, 1, 1).size() < 320);

    lsefit_schedule s{};
    double ms = 0.0;
    CHECK(!tune_cache::lookup(path + ".missing", ka, &s, &ms));   // no file: a miss

    FILE* f = std::fopen(path.c_str(), "w");
    if (!f) return 2;
    std::fprintf(f, "%s\t2048 4 2048 2 0.70\n", ka.c_str());
    std::fprintf(f, "no tab on this line\n");
    std::fprintf(f, "%s extra\t1 1 64 1 9.0\n", ka.c_str());      // longer key: another shape
    std::fprintf(f, "%s\t4096 2 garbage\n", ka.c_str());          // does not parse: skipped
    std::fprintf(f, "%s\t8192 4 256 4 0.65\n", ka.c_str());       // the last parsable line wins
    std::fprintf(f, "%s\n", std::string(1 << 20, 'z').c_str());   // a very long line
    std::fprintf(f, "\t\t\t\n");
    std::fprintf(f, "%s\t", ka.c_str());                          // truncated last line, no newline
    std::fclose(f);

    CHECK(tune_cache::lookup(path, ka, &s, &ms));
    CHECK(s.waves == 8192 && s.waves_per_block == 4 && s.tile == 256 && s.unroll == 4);
    CHECK(ms == 0.65);
    CHECK(!tune_cache::lookup(path, kb, &s, &ms));
    CHECK(!tune_cache::lookup(path, "", &s, &ms));

    // an appended line is found, and wins over the earlier ones
    tune_cache::store(path, kb, lsefit_schedule{1024, 2, 2048, 1}, 0.125);
    tune_cache::store(path, ka, lsefit_schedule{4096, 2, 2048, 2}, 0.5);
    CHECK(tune_cache::lookup(path, kb, &s, &ms));
    CHECK(s.waves == 1024 && s.waves_per_block == 2 && s.tile == 2048 && s.unroll == 1 && ms == 0.125);
    CHECK(tune_cache::lookup(path, ka, &s, &ms));
    CHECK(s.waves == 4096 && s.unroll == 2 && ms == 0.5);
    // the replay form: absent on a line of five fields, 0 or 1 when stored,
    // and absent again when the sixth field is not 0 or 1
    int graph = 7;
    CHECK(tune_cache::lookup(path, ka, &s, &ms, &graph) && graph == -1);
    tune_cache::store(path, ka, lsefit_schedule{2048, 4, 2048, 4}, 0.25, 0);
    CHECK(tune_cache::lookup(path, ka, &s, &ms, &graph) && graph == 0 && s.unroll == 4 && ms == 0.25);
    tune_cache::store(path, ka, lsefit_schedule{2048, 4, 256, 1}, 0.375, 1);
    CHECK(tune_cache::lookup(path, ka, &s, &ms, &graph) && graph == 1 && s.tile == 256 && ms == 0.375);
    tune_cache::store(path, kb, lsefit_schedule{512, 1, 64, 1}, 2.0, 5);   // not a form: not written
    CHECK(tune_cache::lookup(path, kb, &s, &ms, &graph) && graph == -1 && s.waves == 512);
    f = std::fopen(path.c_str(), "a");
    if (!f) return 2;
    std::fprintf(f, "%s\t1024 2 2048 2 0.125 3\n", kb.c_str());
    std::fclose(f);
    CHECK(tune_cache::lookup(path, kb, &s, &ms, &graph) && graph == -1 && s.waves == 1024);
    // a path that cannot be written is left alone
    tune_cache::store(std::string(argv[1]) + "/no/such/dir/cache.txt", ka, s, 1.0);

    if (failures) std::fprintf(stderr, "%d checks failed\n", failures);
    else std::printf("tune cache checks passed\n");
    return failures ? 1 : 0;
}
