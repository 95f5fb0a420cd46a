// Host check of the tile-cache file logic of liblb (lb_tune_cache.hpp):
// store / lookup round trip, several keys in one file, a corrupt file
// ignored and rewritten, every truncation and seeded byte corruptions of a
// valid file read without fault (built with the address and undefined-
// behaviour sanitizers by the test), and the cache switched off.  Prints
// "ok" on success.
//
//     tune_cache_check <cache-file>
#include <cstdint>
#include <cstdio>
#include <cstdlib>

#include "lb_tune_cache.hpp"

static int fails = 0;
#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            std::fprintf(stderr, "check failed: %s\n", #c);       \
            ++fails;                                               \
        }                                                          \
    } while (0)

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    const std::string path = argv[1];
    setenv("LB_TILE_CACHE", path.c_str(), 1);
    lbtune::Choice a, b, got;
    a.spp = 2;
    a.tx = 128;
    a.th = {16, 32};
    a.th2 = {7, 9};
    a.th3 = {12, 16};
    b.spp = 1;
    b.tx = 256;
    b.th = {12};
    b.th2 = {12};
    b.th3 = {10};
    CHECK(!lbtune::lookup("k1", got));
    lbtune::store("gfx950:sramecc+:xnack-|cu256|st0|f0|bc0|spp0|tx0|th0|100x50,100x50", a);
    lbtune::store("k2", b);
    CHECK(lbtune::lookup("gfx950:sramecc+:xnack-|cu256|st0|f0|bc0|spp0|tx0|th0|100x50,100x50", got));
    CHECK(got.spp == 2 && got.tx == 128 && got.th == a.th && got.th2 == a.th2 && got.th3 == a.th3);
    CHECK(lbtune::lookup("k2", got));
    CHECK(got.spp == 1 && got.tx == 256 && got.th == b.th && got.th2 == b.th2 && got.th3 == b.th3);
    CHECK(!lbtune::lookup("k3", got));
    // overwrite a key
    b.tx = 64;
    lbtune::store("k2", b);
    CHECK(lbtune::lookup("k2", got) && got.tx == 64);
    // a corrupt file is ignored, then rewritten by the next store
    FILE *fh = std::fopen(path.c_str(), "wb");
    std::fputs("{\"k2\": {\"spp\": 1, \"tx\": [", fh);
    std::fclose(fh);
    CHECK(!lbtune::lookup("k2", got));
    lbtune::store("k4", a);
    CHECK(lbtune::lookup("k4", got) && got.th == a.th);
    CHECK(!lbtune::lookup("k2", got));
    // every truncation of a valid file, and seeded corruptions of it, are
    // read without fault; a truncated file never yields a choice
    {
        const std::string good = lbtune::to_json({{"k1", a}, {"k2", b}, {"k4", a}});
        for (size_t n = 0; n < good.size(); ++n) {
            std::map<std::string, lbtune::Choice> m;
            const std::string cut = good.substr(0, n);
            const bool ok = lbtune::parse(cut, m);
            // the closing brace is the last non-space character
            CHECK(!ok || cut.find_last_not_of(" \n") == good.find_last_not_of(" \n"));
        }
        uint32_t r = 12345u;
        for (int trial = 0; trial < 20000; ++trial) {
            std::string bad = good;
            for (int k = 0; k < 1 + trial % 4; ++k) {
                r = r * 1664525u + 1013904223u;
                const size_t at = (r >> 8) % bad.size();
                r = r * 1664525u + 1013904223u;
                bad[at] = (char)(r >> 24);
            }
            std::map<std::string, lbtune::Choice> m;
            (void)lbtune::parse(bad, m);
        }
        std::map<std::string, lbtune::Choice> m;
        CHECK(lbtune::parse(good, m) && m.size() == 3 && m["k2"].tx == b.tx);
    }
    // switched off: nothing is read or written
    setenv("LB_TILE_CACHE", "off", 1);
    CHECK(!lbtune::lookup("k4", got));
    lbtune::store("k5", a);
    setenv("LB_TILE_CACHE", path.c_str(), 1);
    CHECK(!lbtune::lookup("k5", got));
    if (fails) return 1;
    std::printf("ok\n");
    return 0;
}
