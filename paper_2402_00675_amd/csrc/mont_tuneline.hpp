// One line of the tuned-shape cache (a JSON object on one line):
//   {"key": "<key>", "<name>": <number>, ...}
// Host-only, with no HIP dependency, so the format is also exercised on the
// CPU.  Numbers are written with 17 significant digits, so every integer
// below 2^53 (tile sizes, grid factors, flags) reads back exactly.
#pragma once

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>

namespace mont {

using TuneRecord = std::map<std::string, double>;

inline std::string tune_format_line(const std::string &key, const TuneRecord &r)
{
    std::string line = "{\"key\": \"" + key + "\"";
    char buf[160];
    for (const auto &kv : r) {
        std::snprintf(buf, sizeof buf, ", \"%s\": %.17g", kv.first.c_str(), kv.second);
        line += buf;
    }
    line += "}\n";
    return line;
}

// Parses a line written by tune_format_line: the key string, then "name":
// number pairs (fields whose value is not a number are skipped).  False when
// the line has no complete "key" string.
inline bool tune_parse_line(const char *s, std::string &key, TuneRecord &r)
{
    const char *k = std::strstr(s, "\"key\"");
    if (!k)
        return false;
    k = std::strchr(k + 5, '"');
    if (!k)
        return false;
    const char *e = std::strchr(k + 1, '"');
    if (!e)
        return false;
    key.assign(k + 1, e);
    r.clear();
    const char *p = e + 1;
    while ((p = std::strchr(p, '"')) != nullptr) {
        const char *q = std::strchr(p + 1, '"');
        if (!q)
            break;
        std::string name(p + 1, q);
        const char *c = q + 1;
        while (*c == ' ' || *c == ':')
            ++c;
        char *end = nullptr;
        const double v = std::strtod(c, &end);
        if (end != c)
            r[name] = v;
        p = end && end != c ? end : q + 1;
    }
    return true;
}

}  // namespace mont
