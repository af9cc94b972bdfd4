// Tuning caches as text (host code): one entry per line, fields separated by
// spaces; the entry kinds and their fields are listed in include/lbm.h
// (lbm_tuning_export).  Each module that keeps a cache exports its entries
// and recognises its own kinds on import.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <string>
#include <vector>

namespace lbm {

inline bool parse_i64(const std::string& t, int64_t& v) {
    if (t.empty()) return false;
    char* end = nullptr;
    const long long x = std::strtoll(t.c_str(), &end, 10);
    if (*end != '\0') return false;
    v = (int64_t)x;
    return true;
}

inline bool parse_f64(const std::string& t, double& v) {
    if (t.empty()) return false;
    char* end = nullptr;
    v = std::strtod(t.c_str(), &end);
    return *end == '\0' && std::isfinite(v);
}

// export appends the module's entries; import returns 1 for a valid entry of
// the module (stored when apply is set), 0 for another module's kind, -1 for
// a malformed entry of the module
void bbatch_tuning_export(std::string& out);
int bbatch_tuning_import(const std::vector<std::string>& f, bool apply);
void abatch_tuning_export(std::string& out);
int abatch_tuning_import(const std::vector<std::string>& f, bool apply);

}  // namespace lbm
