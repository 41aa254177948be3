// Launch-table file: the stored launch geometries of a context, read when
// the context is created and written back when it tunes, so that a tuned
// thread geometry serves later runs (the paper's auto-tuning proposal,
// sections 5.4 and 9).  The file is JSON with a fixed schema:
//   {"device": "gfx950:...", "entries": [
//     {"op": "APE", "prec": "F32", "fmt": "LINK12", "L": [32, 32, 32, 64],
//      "launch": [block, groups_per_wave, xcd_map, t_window, lds_tile]}, ...]}
// (a four-element "launch" leaves lds_tile at -1: the operation's default).
// Entries recorded on another architecture (the part of "device" before the
// first ':') are ignored.  This reader accepts any JSON value where the
// schema does not care (unknown keys are skipped) and rejects everything
// that is not JSON.
#include <cctype>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include <unistd.h>

#include "qdpx_impl.hpp"

namespace qdpx {

namespace {

const char *const kOpNames[] = {"SHIFT", "CHAIN", "APE", "PLAQ", "BATCHED", "JACOBI"};
const char *const kPrecNames[] = {"F64", "F32"};
const char *const kFmtNames[] = {"LINK18", "LINK12"};

template <size_t N> int name_index(const char *const (&names)[N], const std::string &s) {
    for (size_t i = 0; i < N; ++i)
        if (s == names[i]) return (int)i;
    return -1;
}

// Minimal JSON value: enough to walk the schema above.
struct JVal {
    enum Kind { kNull, kBool, kNum, kStr, kArr, kObj } kind = kNull;
    double num = 0.0;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;
    const JVal *get(const char *key) const {
        for (const auto &kv : obj)
            if (kv.first == key) return &kv.second;
        return nullptr;
    }
};

struct Parser {
    const char *p, *end;
    std::string err;
    int depth = 0;

    void ws() {
        while (p < end && (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p;
    }
    bool fail(const char *what) {
        if (err.empty()) err = what;
        return false;
    }
    bool lit(const char *s) {
        const size_t n = strlen(s);
        if ((size_t)(end - p) < n || memcmp(p, s, n) != 0) return fail("unexpected token");
        p += n;
        return true;
    }
    bool string(std::string &out) {
        if (p >= end || *p != '"') return fail("expected a string");
        ++p;
        out.clear();
        while (p < end && *p != '"') {
            char c = *p++;
            if ((unsigned char)c < 0x20) return fail("control character in a string");
            if (c == '\\') {
                if (p >= end) return fail("unterminated escape");
                const char e = *p++;
                switch (e) {
                case '"': case '\\': case '/': out += e; break;
                case 'b': out += '\b'; break;
                case 'f': out += '\f'; break;
                case 'n': out += '\n'; break;
                case 'r': out += '\r'; break;
                case 't': out += '\t'; break;
                case 'u':  // kept as '?': no name in the schema needs it
                    for (int k = 0; k < 4; ++k, ++p)
                        if (p >= end || !isxdigit((unsigned char)*p)) return fail("bad \\u escape");
                    out += '?';
                    break;
                default: return fail("bad escape");
                }
            } else {
                out += c;
            }
        }
        if (p >= end) return fail("unterminated string");
        ++p;
        return true;
    }
    bool number(double &out) {
        const char *s = p;
        if (p < end && *p == '-') ++p;
        if (p >= end || !isdigit((unsigned char)*p)) return fail("bad number");
        while (p < end && (isdigit((unsigned char)*p) || *p == '.' || *p == 'e' || *p == 'E' || *p == '+' ||
                           *p == '-'))
            ++p;
        std::string t(s, p);
        char *q = nullptr;
        out = strtod(t.c_str(), &q);
        if (!q || *q) return fail("bad number");
        return true;
    }
    bool value(JVal &v) {
        if (++depth > 64) return fail("nesting too deep");
        ws();
        if (p >= end) return fail("unexpected end of file");
        bool ok = true;
        if (*p == '{') {
            v.kind = JVal::kObj;
            ++p;
            ws();
            if (p < end && *p == '}') {
                ++p;
            } else {
                for (;;) {
                    ws();
                    std::string k;
                    if (!string(k)) { ok = false; break; }
                    ws();
                    if (p >= end || *p != ':') { ok = fail("expected ':'"); break; }
                    ++p;
                    v.obj.emplace_back(k, JVal());
                    if (!value(v.obj.back().second)) { ok = false; break; }
                    ws();
                    if (p < end && *p == ',') { ++p; continue; }
                    if (p < end && *p == '}') { ++p; break; }
                    ok = fail("expected ',' or '}'");
                    break;
                }
            }
        } else if (*p == '[') {
            v.kind = JVal::kArr;
            ++p;
            ws();
            if (p < end && *p == ']') {
                ++p;
            } else {
                for (;;) {
                    v.arr.emplace_back();
                    if (!value(v.arr.back())) { ok = false; break; }
                    ws();
                    if (p < end && *p == ',') { ++p; continue; }
                    if (p < end && *p == ']') { ++p; break; }
                    ok = fail("expected ',' or ']'");
                    break;
                }
            }
        } else if (*p == '"') {
            v.kind = JVal::kStr;
            ok = string(v.str);
        } else if (*p == 't') {
            v.kind = JVal::kBool;
            v.num = 1;
            ok = lit("true");
        } else if (*p == 'f') {
            v.kind = JVal::kBool;
            ok = lit("false");
        } else if (*p == 'n') {
            ok = lit("null");
        } else {
            v.kind = JVal::kNum;
            ok = number(v.num);
        }
        --depth;
        return ok;
    }
};

std::string arch_base(const std::string &a) { return a.substr(0, a.find(':')); }

// An array of n integers (n in [nmin, nmax]); returns n, or 0 if v is not one.
int int_array(const JVal *v, int *out, int nmin, int nmax) {
    if (!v || v->kind != JVal::kArr || (int)v->arr.size() < nmin || (int)v->arr.size() > nmax) return 0;
    const int n = (int)v->arr.size();
    for (int d = 0; d < n; ++d) {
        const JVal &x = v->arr[d];
        if (x.kind != JVal::kNum || !(x.num > -2147483648.0 && x.num < 2147483648.0) ||
            x.num != (double)(int)x.num)
            return false;
        out[d] = (int)x.num;
    }
    return n;
}

bool int_array4(const JVal *v, int out[4]) { return int_array(v, out, 4, 4) == 4; }

}  // namespace

int tune_table_read(const char *path, const char *arch, std::vector<TuneEntry> &out, std::string &err) {
    out.clear();
    FILE *f = fopen(path, "rb");
    if (!f) {
        if (errno == ENOENT) return 1;
        err = std::string("cannot open ") + path + ": " + strerror(errno);
        return -1;
    }
    std::string text;
    char buf[65536];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) {
        text.append(buf, n);
        if (text.size() > (64u << 20)) {
            fclose(f);
            err = std::string(path) + ": larger than 64 MiB";
            return -1;
        }
    }
    const bool rerr = ferror(f) != 0;
    fclose(f);
    if (rerr) {
        err = std::string("cannot read ") + path;
        return -1;
    }
    Parser ps{text.data(), text.data() + text.size()};
    JVal root;
    if (!ps.value(root)) {
        err = std::string(path) + ": not JSON (" + ps.err + " at byte " + std::to_string(ps.p - text.data()) + ")";
        return -1;
    }
    ps.ws();
    if (ps.p != ps.end) {
        err = std::string(path) + ": trailing characters after the JSON value";
        return -1;
    }
    const JVal *dev = root.kind == JVal::kObj ? root.get("device") : nullptr;
    const JVal *ents = root.kind == JVal::kObj ? root.get("entries") : nullptr;
    if (!dev || dev->kind != JVal::kStr || !ents || ents->kind != JVal::kArr) {
        err = std::string(path) + ": expected an object with a \"device\" string and an \"entries\" array";
        return -1;
    }
    if (arch_base(dev->str) != arch_base(arch)) return 2;  // recorded on another architecture
    for (size_t i = 0; i < ents->arr.size(); ++i) {
        const JVal &e = ents->arr[i];
        const JVal *op = e.get("op"), *prec = e.get("prec"), *fmt = e.get("fmt");
        TuneEntry t;
        int launch[5] = {0, 0, 0, 0, -1};  // a table without the LDS tile field: -1, the default
        const bool ok = e.kind == JVal::kObj && op && op->kind == JVal::kStr && prec && prec->kind == JVal::kStr &&
                        fmt && fmt->kind == JVal::kStr && int_array4(e.get("L"), t.L) &&
                        int_array(e.get("launch"), launch, 4, 5) > 0 && (t.op = name_index(kOpNames, op->str)) >= 0 &&
                        (t.prec = name_index(kPrecNames, prec->str)) >= 0 &&
                        (t.fmt = name_index(kFmtNames, fmt->str)) >= 0;
        if (!ok) {
            err = std::string(path) + ": entry " + std::to_string(i) + " does not have the expected fields";
            out.clear();
            return -1;
        }
        t.cfg.block = launch[0];
        t.cfg.nsite = launch[1];
        t.cfg.xcd = launch[2];
        t.cfg.tw = launch[3];
        t.cfg.lds = launch[4];
        out.push_back(t);
    }
    return 0;
}

int tune_table_write(const char *path, const char *arch, const std::vector<TuneEntry> &in, std::string &err) {
    std::string s = "{\n \"device\": \"";
    for (const char *c = arch; *c; ++c)
        if (*c != '"' && *c != '\\' && (unsigned char)*c >= 0x20) s += *c;
    s += "\",\n \"entries\": [";
    bool first = true;
    for (const TuneEntry &t : in) {
        if (t.op < 0 || t.op >= 6 || t.prec < 0 || t.prec >= 2 || t.fmt < 0 || t.fmt >= 2) continue;
        char line[256];
        snprintf(line, sizeof line,
                 "%s\n  {\"op\": \"%s\", \"prec\": \"%s\", \"fmt\": \"%s\", \"L\": [%d, %d, %d, %d], "
                 "\"launch\": [%d, %d, %d, %d, %d]}",
                 first ? "" : ",", kOpNames[t.op], kPrecNames[t.prec], kFmtNames[t.fmt], t.L[0], t.L[1], t.L[2], t.L[3],
                 t.cfg.block, t.cfg.nsite, t.cfg.xcd, t.cfg.tw, t.cfg.lds);
        s += line;
        first = false;
    }
    s += "\n ]\n}\n";
    // write a private temporary file next to the target, then rename it into
    // place, so a reader never sees a partial table
    std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) {
        err = "cannot create " + tmp + ": " + strerror(errno);
        return -1;
    }
    const bool wok = fwrite(s.data(), 1, s.size(), f) == s.size();
    const bool cok = fclose(f) == 0;
    if (!wok || !cok || rename(tmp.c_str(), path) != 0) {
        err = std::string("cannot write ") + path + ": " + strerror(errno);
        (void)remove(tmp.c_str());
        return -1;
    }
    return 0;
}

}  // namespace qdpx
