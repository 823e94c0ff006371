// Host-only driver for the tuned-table reader (paper_1304_7053_amd/csrc/
// tuned_table.cpp), built with AddressSanitizer and UndefinedBehaviorSanitizer
// by tests/test_tuned_table_fuzz.py.  The reader parses a file the user can
// point the library at (SBG_TUNE_FILE), so it must survive any bytes: every
// prefix of a valid table, seeded random mutations of it, and hand-written
// hostile inputs (deep nesting, numbers outside int's range, NaN, unterminated
// strings, stray escapes, NUL bytes).  Any memory error or undefined behaviour
// aborts the run; the driver also checks what a valid table and a few
// malformed ones parse to.  Prints "fuzz ok <cases>" on success.
#include "tuned_table.cpp"

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

namespace {

int count_of(const std::string& text)
{
    sbg::Table t;
    std::memset(t.has, 0, sizeof(t.has));
    t.count = 0;
    t.version = 0;
    sbg::parse(text, t);
    return t.version == 1 ? t.count : -1;
}

std::string valid_table()
{
    return "{\"version\": 1, \"library\": \"libsbg\", \"entries\": ["
           "{\"type\": \"s\", \"form\": \"strided\", \"ops\": \"NN\", \"size\": 5, \"path\": \"team\", "
           "\"unroll\": 0, \"wg_per_cu\": 0, \"xcd_chunk\": 0, \"us\": 13.3, \"paths_us\": {\"mfma\": 22.0}},"
           "{\"type\": \"d\", \"form\": \"pointer\", \"ops\": \"TN\", \"size\": 16, \"path\": \"mfma\", "
           "\"unroll\": 2, \"wg_per_cu\": 4, \"xcd_chunk\": 16, \"note\": \"a \\\"quoted\\\" word\"}"
           "], \"grid_sweep\": [{\"points\": [{\"work_groups\": 8, \"us\": 1.5e3}, [true, false, null]]}]}";
}

uint64_t lcg(uint64_t& s)
{
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return s >> 33;
}

}  // namespace

int main()
{
    long cases = 0;
    const std::string good = valid_table();
    if (count_of(good) != 2) {
        std::printf("valid table: %d entries, want 2\n", count_of(good));
        return 1;
    }
    // every prefix (truncated files)
    for (size_t n = 0; n <= good.size(); ++n, ++cases) count_of(good.substr(0, n));
    // seeded mutations: replace, insert or delete a few bytes
    uint64_t seed = 13047053;
    const char alphabet[] = "{}[]:,\"\\-+.0123456789eEtfn \t\nxyz\x01\xff";
    for (int it = 0; it < 20000; ++it, ++cases) {
        std::string s = good;
        const int edits = 1 + (int)(lcg(seed) % 4);
        for (int e = 0; e < edits && !s.empty(); ++e) {
            const size_t pos = lcg(seed) % s.size();
            const char c = alphabet[lcg(seed) % (sizeof(alphabet) - 1)];
            switch (lcg(seed) % 3) {
                case 0: s[pos] = c; break;
                case 1: s.insert(s.begin() + (long)pos, c); break;
                default: s.erase(pos, 1); break;
            }
        }
        count_of(s);
    }
    // hostile inputs
    const std::vector<std::string> hostile = {
        "", " ", "{", "}", "[", "\"", "{\"", "{\"version\"", "{\"version\":", "{\"version\": 1",
        "{\"version\": 1e400, \"entries\": []}",
        "{\"version\": -1e30, \"entries\": []}",
        "{\"version\": nan, \"entries\": []}",
        "{\"version\": 1, \"entries\": [{\"type\": \"s\", \"form\": \"strided\", \"ops\": \"NN\", \"size\": 1e300}]}",
        "{\"version\": 1, \"entries\": [{\"type\": \"s\", \"form\": \"strided\", \"ops\": \"NN\", \"size\": -9e18}]}",
        "{\"version\": 1, \"entries\": [{\"type\": \"s\", \"form\": \"strided\", \"ops\": \"NN\", \"size\": 4, "
        "\"unroll\": 1e99, \"wg_per_cu\": -1e99, \"xcd_chunk\": 4294967296}]}",
        "{\"version\": 1, \"entries\": [{\"type\": \"s\", \"form\": \"strided\", \"ops\": \"N\", \"size\": 4}]}",
        "{\"version\": 1, \"entries\": [{\"ops\": \"\\",
        "{\"version\": 1, \"x\": \"unterminated",
        std::string("{\"version\": 1, \"x\": \"a\0b\", \"entries\": []}", 40),
        std::string(100000, '['),
        std::string(100000, '{'),
        "{\"version\": 1, \"x\": " + std::string(5000, '[') + std::string(5000, ']') + ", \"entries\": []}",
        "{\"version\": 1, \"entries\": [" + std::string(3000, ',') + "]}",
    };
    for (const std::string& h : hostile) {
        count_of(h);
        ++cases;
    }
    // what a few of them must parse to
    if (count_of("{\"version\": 1e400, \"entries\": []}") != -1) return 2;
    if (count_of("{\"version\": 1, \"entries\": [{\"type\": \"s\", \"form\": \"strided\", \"ops\": \"NN\", "
                 "\"size\": 1e300}]}") != 0)
        return 3;
    if (count_of(std::string(100000, '[')) != -1) return 4;
    if (count_of("{\"version\": 1, \"x\": " + std::string(5000, '[') + std::string(5000, ']') +
                 ", \"entries\": []}") != -1)
        return 5;   // nesting beyond the reader's limit fails the read
    if (count_of("{\"version\": 1, \"x\": [[[1]]], \"entries\": []}") != 0) return 6;
    std::printf("fuzz ok %ld\n", cases);
    return 0;
}
