// The autotuner's choices as a JSON file, so that a later process on the same kind of GPU and
// the same HIP runtime starts from them instead of timing again.  Host-only and free of HIP,
// so that a CPU test (under the sanitizers) covers the writer, the reader and its rejection of
// malformed files.
//
// Format (one object; keys in any order, whitespace free):
//   {"format": "zoneburn-tune-1", "arch": "<gcnArchName>", "hip_runtime": <int>,
//    "entries": [{"nv": 14, "nr": 30, "precision": 1, "lanes": 16,
//                 "auto_lanes": 16, "auto_lu": 0}, ...]}
// An entry is keyed by (nv, nr, precision); lanes is the mapping with the vector LU, and
// (auto_lanes, auto_lu) the pair for ZB_LU_AUTO.
#pragma once

#include <stdint.h>
#include <stdio.h>

#include <map>
#include <memory>
#include <string>
#include <vector>

namespace zbh {

struct TuneEntry {
    int nv, nr, prec, lanes, auto_lanes, auto_lu;
};

inline std::string tune_json(const std::string &arch, int runtime, const std::vector<TuneEntry> &es)
{
    std::string s = "{\"format\": \"zoneburn-tune-1\", \"arch\": \"";
    for (char ch : arch) {   // the architecture name is plain ASCII; anything else is dropped
        if (ch == '"' || ch == '\\' || (unsigned char)ch < 0x20 || (unsigned char)ch > 0x7e) continue;
        s += ch;
    }
    s += "\", \"hip_runtime\": " + std::to_string(runtime) + ", \"entries\": [";
    for (size_t i = 0; i < es.size(); ++i) {
        const TuneEntry &e = es[i];
        char b[192];
        snprintf(b, sizeof b,
                 "%s\n  {\"nv\": %d, \"nr\": %d, \"precision\": %d, \"lanes\": %d, "
                 "\"auto_lanes\": %d, \"auto_lu\": %d}",
                 i ? "," : "", e.nv, e.nr, e.prec, e.lanes, e.auto_lanes, e.auto_lu);
        s += b;
    }
    s += "\n]}\n";
    return s;
}

// A small JSON reader: objects, arrays, strings (escapes \" \\ \/ \b \f \n \r \t; \u is
// refused), integers, true/false/null.  Fractions and exponents are refused: the format has
// none.  Depth is bounded.
struct JVal {
    enum Kind { NUL, BOOL, INT, STR, ARR, OBJ } kind = NUL;
    bool b = false;
    long long i = 0;
    std::string s;
    std::vector<JVal> a;
    std::map<std::string, JVal> o;
};

class JReader {
  public:
    explicit JReader(const std::string &t) : t_(t) {}
    bool parse(JVal &v, std::string &err)
    {
        if (!value(v, 0)) {
            err = err_.empty() ? "malformed JSON" : err_;
            return false;
        }
        ws();
        if (p_ != t_.size()) {
            err = "trailing characters after the JSON value";
            return false;
        }
        return true;
    }

  private:
    const std::string &t_;
    size_t p_ = 0;
    std::string err_;

    void ws()
    {
        while (p_ < t_.size() && (t_[p_] == ' ' || t_[p_] == '\t' || t_[p_] == '\n' || t_[p_] == '\r')) ++p_;
    }
    bool lit(const char *w)
    {
        size_t n = 0;
        while (w[n]) ++n;
        if (t_.compare(p_, n, w) != 0) return false;
        p_ += n;
        return true;
    }
    bool str(std::string &out)
    {
        if (p_ >= t_.size() || t_[p_] != '"') return false;
        ++p_;
        while (p_ < t_.size()) {
            const char ch = t_[p_++];
            if (ch == '"') return true;
            if ((unsigned char)ch < 0x20) return false;
            if (ch != '\\') {
                out += ch;
                continue;
            }
            if (p_ >= t_.size()) return false;
            const char e = t_[p_++];
            switch (e) {
            case '"': out += '"'; break;
            case '\\': out += '\\'; break;
            case '/': out += '/'; break;
            case 'b': out += '\b'; break;
            case 'f': out += '\f'; break;
            case 'n': out += '\n'; break;
            case 'r': out += '\r'; break;
            case 't': out += '\t'; break;
            default: err_ = "unsupported string escape"; return false;
            }
        }
        return false;
    }
    bool num(long long &out)
    {
        size_t q = p_;
        bool neg = false;
        if (q < t_.size() && t_[q] == '-') {
            neg = true;
            ++q;
        }
        if (q >= t_.size() || t_[q] < '0' || t_[q] > '9') return false;
        long long v = 0;
        while (q < t_.size() && t_[q] >= '0' && t_[q] <= '9') {
            if (v > (1LL << 40)) {   // far beyond any field of the format
                err_ = "number out of range";
                return false;
            }
            v = v * 10 + (t_[q] - '0');
            ++q;
        }
        if (q < t_.size() && (t_[q] == '.' || t_[q] == 'e' || t_[q] == 'E')) {
            err_ = "non-integer number";
            return false;
        }
        p_ = q;
        out = neg ? -v : v;
        return true;
    }
    bool value(JVal &v, int depth)
    {
        if (depth > 8) {
            err_ = "nesting too deep";
            return false;
        }
        ws();
        if (p_ >= t_.size()) return false;
        const char ch = t_[p_];
        if (ch == '{') {
            ++p_;
            v.kind = JVal::OBJ;
            ws();
            if (p_ < t_.size() && t_[p_] == '}') {
                ++p_;
                return true;
            }
            for (;;) {
                ws();
                std::string k;
                if (!str(k)) return false;
                ws();
                if (p_ >= t_.size() || t_[p_] != ':') return false;
                ++p_;
                JVal x;
                if (!value(x, depth + 1)) return false;
                if (v.o.count(k)) {
                    err_ = "duplicate key " + k;
                    return false;
                }
                v.o.emplace(k, std::move(x));
                ws();
                if (p_ < t_.size() && t_[p_] == ',') {
                    ++p_;
                    continue;
                }
                if (p_ < t_.size() && t_[p_] == '}') {
                    ++p_;
                    return true;
                }
                return false;
            }
        }
        if (ch == '[') {
            ++p_;
            v.kind = JVal::ARR;
            ws();
            if (p_ < t_.size() && t_[p_] == ']') {
                ++p_;
                return true;
            }
            for (;;) {
                JVal x;
                if (!value(x, depth + 1)) return false;
                v.a.push_back(std::move(x));
                ws();
                if (p_ < t_.size() && t_[p_] == ',') {
                    ++p_;
                    continue;
                }
                if (p_ < t_.size() && t_[p_] == ']') {
                    ++p_;
                    return true;
                }
                return false;
            }
        }
        if (ch == '"') {
            v.kind = JVal::STR;
            return str(v.s);
        }
        if (lit("true")) {
            v.kind = JVal::BOOL;
            v.b = true;
            return true;
        }
        if (lit("false")) {
            v.kind = JVal::BOOL;
            return true;
        }
        if (lit("null")) return true;
        v.kind = JVal::INT;
        return num(v.i);
    }
};

// Reads a file written by tune_json.  Entries must have every field, as integers in range:
// nv 1..nv_max, nr 0..nr_max, precision 0/1, lanes and auto_lanes powers of two 1..64,
// auto_lu 0/1; any other content is an error (err says which).
inline bool tune_parse(const std::string &text, int nv_max, int nr_max, std::string &arch,
                       int &runtime, std::vector<TuneEntry> &out, std::string &err)
{
    JVal root;
    JReader rd(text);
    if (!rd.parse(root, err)) return false;
    if (root.kind != JVal::OBJ) {
        err = "not a JSON object";
        return false;
    }
    auto field = [&](const JVal &o, const char *k, JVal::Kind kind) -> const JVal * {
        auto it = o.o.find(k);
        if (it == o.o.end() || it->second.kind != kind) {
            err = std::string("missing or mistyped field ") + k;
            return nullptr;
        }
        return &it->second;
    };
    const JVal *fmt = field(root, "format", JVal::STR);
    if (!fmt) return false;
    if (fmt->s != "zoneburn-tune-1") {
        err = "unknown format " + fmt->s;
        return false;
    }
    const JVal *a = field(root, "arch", JVal::STR);
    const JVal *rt = a ? field(root, "hip_runtime", JVal::INT) : nullptr;
    const JVal *es = rt ? field(root, "entries", JVal::ARR) : nullptr;
    if (!es) return false;
    if (rt->i < 0 || rt->i > 0x7fffffff) {
        err = "hip_runtime out of range";
        return false;
    }
    auto pow2 = [](long long v) { return v >= 1 && v <= 64 && (v & (v - 1)) == 0; };
    std::vector<TuneEntry> got;
    for (const JVal &e : es->a) {
        if (e.kind != JVal::OBJ) {
            err = "an entry is not an object";
            return false;
        }
        const char *names[6] = {"nv", "nr", "precision", "lanes", "auto_lanes", "auto_lu"};
        long long v[6];
        for (int i = 0; i < 6; ++i) {
            const JVal *f = field(e, names[i], JVal::INT);
            if (!f) return false;
            v[i] = f->i;
        }
        if (e.o.size() != 6) {
            err = "an entry has unknown fields";
            return false;
        }
        if (v[0] < 1 || v[0] > nv_max || v[1] < 0 || v[1] > nr_max || (v[2] != 0 && v[2] != 1) ||
            !pow2(v[3]) || !pow2(v[4]) || (v[5] != 0 && v[5] != 1)) {
            err = "an entry's values are out of range";
            return false;
        }
        got.push_back({(int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4], (int)v[5]});
    }
    arch = a->s;
    runtime = (int)rt->i;
    out.swap(got);
    return true;
}

}  // namespace zbh
