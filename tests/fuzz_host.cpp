// Seeded fuzz of the library's host-only logic (admm_host.cpp), built with the
// address and undefined-behaviour sanitizers by tests/test_host_sanitizers.py:
// the tuning-cache parser on malformed and mutated text, the cache file round
// trip, the cache key, and the plan-time validation of random problems. Any
// out-of-bounds access, overflow or invalid conversion aborts the run; the
// checks below also fail it on a wrong answer.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <map>
#include <random>
#include <string>
#include <vector>

#include "../paper_1210_2687_amd/csrc/admm_host.h"

using namespace admm_host;

static int failures = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++failures;                                                  \
        }                                                                \
    } while (0)

int main(int argc, char** argv) {
    const char* dir = argc > 1 ? argv[1] : ".";
    std::mt19937_64 g(12345);
    // ---- cache text: fixed malformed cases
    const char* bad[] = {"", "{", "}", "{\"a\"", "{\"a\":", "{\"a\":{", "{\"a\":{\"tc\":}}", "{\"a\":{\"tc\":1,}}",
                         "{\"a\":{\"tc\":1e999}}", "{\"a\":{\"tc\":-3}}", "{\"a\":{\"rows\":nan}}",
                         "{\"a\":{\"rows\":1e300}}", "{\"a\":{\"tc\":2.5}}", "{\"a\":{\"col_us\":-1}}",
                         "{\"a\":{\"col_us\":inf}}", "{\"a\\\"\":{}}", "{\"a\":{\"tc\":1}", "[1,2]",
                         "{\"a\":{\"tc\":2147483648}}", "{\"a\":{\"tc\":-2147483649}}", "{\"\":{\"\":0}} x",
                         "{\"a\":{\"rsched\":4}}", "{\"a\":{\"csched\":1.5}}"};
    for (const char* t : bad) {
        std::map<std::string, TuneEntry> m;
        CHECK(!parse_cache(t, m));
    }
    // ---- a valid cache, its round trip, and random mutations of it
    std::map<std::string, TuneEntry> ref;
    for (int i = 0; i < 40; ++i) {
        TuneEntry e;
        e.tc = 1 + (int)(g() % 4);
        e.rows = 1 + (int)(g() % 16);
        e.rows_c[g() % admm_host::kRowClasses] = (int)(g() % 17);
        e.rsched = (int)(g() % 4);
        e.csched = (int)(g() % 3);
        e.col_us = (double)(g() % 100000) / 1000.0;
        e.row_us = (double)(g() % 100000) / 1000.0;
        ref["gfx950|tv" + std::to_string(i) + "x" + std::to_string(g() % 2048) + "*8"] = e;
    }
    const std::string text = format_cache(ref);
    std::map<std::string, TuneEntry> back;
    CHECK(parse_cache(text, back));
    CHECK(back.size() == ref.size());
    for (const auto& kv : ref) {
        const auto it = back.find(kv.first);
        CHECK(it != back.end() && it->second.tc == kv.second.tc && it->second.rows == kv.second.rows &&
              it->second.rows_c[0] == kv.second.rows_c[0] && it->second.rows_c[1] == kv.second.rows_c[1] &&
              it->second.rows_c[2] == kv.second.rows_c[2] && it->second.rows_c[3] == kv.second.rows_c[3] &&
              it->second.rows_c[4] == kv.second.rows_c[4] &&
              it->second.rsched == kv.second.rsched &&
              it->second.csched == kv.second.csched);
    }
    const char alphabet[] = "{}[]\":,. -+0123456789eEinfatcrowsu_x\\\n\t";
    long parsed = 0;
    for (int it = 0; it < 20000; ++it) {
        std::string t = text;
        const int edits = 1 + (int)(g() % 8);
        for (int e = 0; e < edits && !t.empty(); ++e) {
            const size_t pos = g() % (t.size() + 1);
            switch (g() % 4) {
                case 0: t.insert(t.begin() + pos, alphabet[g() % (sizeof alphabet - 1)]); break;
                case 1: if (pos < t.size()) t.erase(pos, 1 + g() % 4); break;
                case 2: if (pos < t.size()) t[pos] = alphabet[g() % (sizeof alphabet - 1)]; break;
                default: t = t.substr(0, pos); break;
            }
        }
        std::map<std::string, TuneEntry> m;
        if (parse_cache(t, m)) {
            ++parsed;
            for (const auto& kv : m) {
                CHECK(kv.second.tc >= 0 && kv.second.tc <= (int)kMaxTileCount);
                CHECK(kv.second.rows >= 0 && kv.second.rows <= (int)kMaxTileCount);
                CHECK(std::isfinite(kv.second.col_us) && kv.second.col_us >= 0.0);
                CHECK(kv.second.rsched >= 0 && kv.second.rsched < kScheduleVariants);
            }
        }
    }
    // ---- random bytes
    for (int it = 0; it < 5000; ++it) {
        std::string t(g() % 200, '\0');
        for (auto& c : t) c = (char)(g() & 0xff);
        if (g() % 2) t[0] = '{';
        std::map<std::string, TuneEntry> m;
        (void)parse_cache(t, m);
    }
    // ---- file round trip
    const std::string path = std::string(dir) + "/fuzz_cache.json";
    CHECK(write_cache(path.c_str(), ref) == 0);
    std::map<std::string, TuneEntry> rd;
    CHECK(read_cache(path.c_str(), rd) == 0 && rd.size() == ref.size());
    std::map<std::string, TuneEntry> none;
    CHECK(read_cache((std::string(dir) + "/absent.json").c_str(), none) == 0 && none.empty());
    FILE* f = std::fopen(path.c_str(), "wb");
    std::fputs("{\"k\": {\"tc\": 3", f);
    std::fclose(f);
    CHECK(read_cache(path.c_str(), rd) == -1);
    // ---- validation of random problems (host pointers only)
    std::vector<float> kern(31 * 31), mask_dummy(1);
    uint8_t mask_byte = 1;
    long ok = 0;
    for (int it = 0; it < 20000; ++it) {
        admm_problem p{};
        const int pick = (int)(g() % 6);
        p.H = pick == 0 ? (int)(g() % 5000) - 100 : (int)(8 + g() % 2041);
        p.W = pick == 1 ? std::numeric_limits<int>::max() - (int)(g() % 3) : (int)(8 + g() % 2041);
        p.ksize = pick == 2 ? (int)(g() % 100) - 50 : 1 + 2 * (int)(g() % 16);
        for (int i = 0; i < p.ksize * p.ksize && p.ksize > 0 && i < (int)kern.size(); ++i)
            kern[i] = (float)((double)(g() % 2001) / 1000.0 - 1.0);
        if (g() % 50 == 0) kern[g() % kern.size()] = std::numeric_limits<float>::quiet_NaN();
        p.kernel = (g() % 40 == 0 || p.ksize > 31) ? nullptr : kern.data();
        p.mask = g() % 40 == 0 ? nullptr : &mask_byte;
        p.reg = (int)(g() % 3) - (g() % 10 == 0 ? 5 : 0);
        p.levels = (int)(g() % 7) - 1;
        const double lams[] = {1e-3, 0.0, -1.0, std::numeric_limits<double>::infinity(),
                               std::numeric_limits<double>::quiet_NaN(), 1e300};
        p.lambda = lams[g() % 6];
        p.mu1 = g() % 7 == 0 ? std::numeric_limits<double>::quiet_NaN() : 1e-3;
        p.mu2 = 1e-3;
        const admm_status s = validate(p);
        CHECK(s >= ADMM_OK && s <= ADMM_E_DIVERGED);
        if (s == ADMM_OK) {
            ++ok;
            CHECK(smooth7(p.H) && smooth7(p.W) && p.ksize % 2 == 1 && p.kernel && p.mask);
        } else {
            CHECK(last_error()[0] != '\0');
        }
    }
    // ---- cache keys, short and hashed
    std::vector<admm_problem> batch(300);
    for (auto& p : batch) {
        p.H = 8 + (int)(g() % 2041);
        p.W = 8 + (int)(g() % 2041);
        p.reg = (int)(g() % 2);
        p.levels = 1 + (int)(g() % 4);
    }
    for (int n : {1, 3, 300}) {
        const std::string k = make_key(batch.data(), n, "gfx950");
        CHECK(k.rfind("gfx950|", 0) == 0 && k.size() < 200);
    }
    std::printf("fuzz_host: %ld mutated caches parsed, %ld valid problems, %d failures\n", parsed, ok, failures);
    return failures == 0 ? 0 : 1;
}
