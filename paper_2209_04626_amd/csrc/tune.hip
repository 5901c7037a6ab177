// Tuning table: Jacobi block widths per problem size and the persistent
// grid of the batched kernel, measured by the autotuner
// (paper_2209_04626_amd/autotune.py) on the target GPU and handed to the
// library as JSON text:
//
//   {"arch": "gfx950",
//    "single":  [{"nmax": 128, "b_low": 16, "b_work": 16}, ...],
//    "batched": [{"nmax": 256, "wg_per_cu": 2}, ...]}
//
// An entry applies to problems with n <= nmax (the smallest such nmax wins).
// Host code only; the table is read under a mutex and copied on lookup.
#include <algorithm>
#include <cctype>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mpjsvd.h"
#include "internal.hpp"

namespace mpj {
namespace {

struct SingleEntry { int nmax, b_low, b_work; };
struct BatchedEntry { int nmax, wg_per_cu; };

std::mutex g_mu;
std::vector<SingleEntry> g_single;
std::vector<BatchedEntry> g_batched;

// A small JSON reader: objects, arrays, numbers, strings, true/false/null.
// Only what the table needs is kept: for each object inside the "single" and
// "batched" arrays, its integer-valued members.
struct Reader {
    const char *p, *end;
    bool ok = true;
    void ws() { while (p < end && std::isspace((unsigned char)*p)) ++p; }
    bool eat(char c) { ws(); if (p < end && *p == c) { ++p; return true; } return false; }
    bool string(std::string *out) {
        ws();
        if (p >= end || *p != '"') return ok = false;
        ++p;
        std::string s;
        while (p < end && *p != '"') {
            if (*p == '\\') { ++p; if (p >= end) return ok = false; }
            s.push_back(*p++);
        }
        if (p >= end) return ok = false;
        ++p;
        if (out) *out = s;
        return true;
    }
    bool number(double *out) {
        ws();
        char *e = nullptr;
        const double v = std::strtod(p, &e);
        if (e == p || e > end) return ok = false;
        p = e;
        if (out) *out = v;
        return true;
    }
    // skip any value
    bool value() {
        ws();
        if (p >= end) return ok = false;
        if (*p == '{') {
            ++p;
            if (eat('}')) return true;
            do {
                if (!string(nullptr) || !eat(':') || !value()) return ok = false;
            } while (eat(','));
            return eat('}') || (ok = false);
        }
        if (*p == '[') {
            ++p;
            if (eat(']')) return true;
            do { if (!value()) return ok = false; } while (eat(','));
            return eat(']') || (ok = false);
        }
        if (*p == '"') return string(nullptr);
        for (const char *lit : {"true", "false", "null"}) {
            const size_t l = std::strlen(lit);
            if ((size_t)(end - p) >= l && std::strncmp(p, lit, l) == 0) { p += l; return true; }
        }
        return number(nullptr);
    }
    // an object of scalar members -> (name, number) pairs
    bool flat_object(std::vector<std::pair<std::string, double>> *kv) {
        if (!eat('{')) return ok = false;
        if (eat('}')) return true;
        do {
            std::string k;
            if (!string(&k) || !eat(':')) return ok = false;
            ws();
            if (p < end && (*p == '-' || std::isdigit((unsigned char)*p))) {
                double v;
                if (!number(&v)) return false;
                kv->push_back({k, v});
            } else if (!value()) {
                return false;
            }
        } while (eat(','));
        return eat('}') || (ok = false);
    }
};

int member(const std::vector<std::pair<std::string, double>> &kv, const char *name) {
    for (auto &e : kv)
        if (e.first == name) return (int)e.second;
    return 0;
}

} // namespace

int tuned_block_cols(int n, bool low) {
    std::lock_guard<std::mutex> lk(g_mu);
    int best = -1, bn = 0;
    for (auto &e : g_single)
        if (n <= e.nmax && (best < 0 || e.nmax < bn)) { best = low ? e.b_low : e.b_work; bn = e.nmax; }
    return best < 0 ? 0 : best;
}

int tuned_wg_per_cu(int nmax) {
    std::lock_guard<std::mutex> lk(g_mu);
    int best = -1, bn = 0;
    for (auto &e : g_batched)
        if (nmax <= e.nmax && (best < 0 || e.nmax < bn)) { best = e.wg_per_cu; bn = e.nmax; }
    return best < 0 ? 0 : best;
}

} // namespace mpj

using namespace mpj;

extern "C" int svd_set_tuning(const char *json) {
    if (!json) {
        std::lock_guard<std::mutex> lk(g_mu);
        g_single.clear();
        g_batched.clear();
        return 0;
    }
    Reader r{json, json + std::strlen(json)};
    std::vector<SingleEntry> single;
    std::vector<BatchedEntry> batched;
    if (!r.eat('{')) return -2;
    if (!r.eat('}')) {
        do {
            std::string key;
            if (!r.string(&key) || !r.eat(':')) return -2;
            if (key == "single" || key == "batched") {
                if (!r.eat('[')) return -2;
                if (!r.eat(']')) {
                    do {
                        std::vector<std::pair<std::string, double>> kv;
                        if (!r.flat_object(&kv)) return -2;
                        const int nmax = member(kv, "nmax");
                        if (nmax < 1) return -3;
                        if (key == "single") {
                            const int bl = member(kv, "b_low"), bw = member(kv, "b_work");
                            if ((bl != 16 && bl != 32) || (bw != 16 && bw != 32)) return -3;
                            single.push_back({nmax, bl, bw});
                        } else {
                            const int w = member(kv, "wg_per_cu");
                            if (w < 1 || w > 16) return -3;
                            batched.push_back({nmax, w});
                        }
                    } while (r.eat(','));
                    if (!r.eat(']')) return -2;
                }
            } else if (!r.value()) {
                return -2;
            }
        } while (r.eat(','));
        if (!r.eat('}')) return -2;
    }
    if (!r.ok) return -2;
    std::lock_guard<std::mutex> lk(g_mu);
    g_single = single;
    g_batched = batched;
    return 0;
}

extern "C" int svd_tuning_lookup(int n, int *b_low, int *b_work, int *wg_per_cu) {
    const int bl = tuned_block_cols(n, true), bw = tuned_block_cols(n, false);
    const int w = tuned_wg_per_cu(n);
    if (b_low) *b_low = bl;
    if (b_work) *b_work = bw;
    if (wg_per_cu) *wg_per_cu = w;
    return (bl || bw || w) ? 1 : 0;
}
