// CPU checks of the tuned-shape cache line format (mont_tuneline.hpp): round
// trips, exact integers, tolerated spacing, skipped non-numeric fields and
// rejected lines.  Prints one line per failed check; exit status = failures.
#include <cmath>
#include <cstdio>

#include "../../paper_2402_00675_amd/csrc/mont_tuneline.hpp"

using mont::TuneRecord;

static int fails = 0;

static void expect(bool ok, const char *what)
{
    if (!ok) {
        std::printf("FAIL %s\n", what);
        ++fails;
    }
}

static bool same(const TuneRecord &a, const TuneRecord &b)
{
    if (a.size() != b.size())
        return false;
    for (const auto &kv : a) {
        auto it = b.find(kv.first);
        if (it == b.end() || it->second != kv.second)
            return false;
    }
    return true;
}

int main()
{
    std::string key;
    TuneRecord r;
    // round trip, exact for integers and doubles
    const TuneRecord rec = {{"tile_elems", 16384}, {"blocks_per_cu", 2}, {"dynamic", 8}, {"nontemporal", 1},
                            {"block", 256}, {"ms", 0.0012345678901234567}, {"big", 1048576},
                            {"huge", 4503599627370497.0}};
    const std::string k0 = "gfx950:v65539:ragged:n4096:log2e28:ops1";
    const std::string line = mont::tune_format_line(k0, rec);
    expect(line.back() == '\n' && line.find('\n') == line.size() - 1, "one line");
    expect(mont::tune_parse_line(line.c_str(), key, r), "parse own line");
    expect(key == k0, "key round trip");
    expect(same(r, rec), "record round trip");
    // spacing variants and an empty record
    expect(mont::tune_parse_line("{ \"key\" :  \"a:b\" ,\"x\":3,  \"y\" :  -2.5 }", key, r) && key == "a:b" &&
               r.size() == 2 && r["x"] == 3 && r["y"] == -2.5,
           "spacing");
    expect(mont::tune_parse_line("{\"key\": \"only\"}", key, r) && key == "only" && r.empty(), "empty record");
    // fields that are not numbers are skipped, numbers after them still read
    expect(mont::tune_parse_line("{\"key\": \"k\", \"note\": \"text\", \"a\": 7}", key, r) && r.size() == 1 &&
               r["a"] == 7,
           "non-numeric field");
    // a later parse starts from an empty record
    expect(mont::tune_parse_line("{\"key\": \"k2\", \"b\": 1}", key, r) && r.size() == 1 && r.count("b"),
           "record cleared");
    // lines without a complete key are rejected
    expect(!mont::tune_parse_line("{\"unroll\": 2}", key, r), "no key");
    expect(!mont::tune_parse_line("{\"key\": \"unterminated", key, r), "unterminated key");
    expect(!mont::tune_parse_line("", key, r), "empty line");
    // a truncated record keeps the fields read so far
    expect(mont::tune_parse_line("{\"key\": \"t\", \"a\": 5, \"b", key, r) && r.size() == 1 && r["a"] == 5,
           "truncated");
    std::printf("%d failures\n", fails);
    return fails;
}
