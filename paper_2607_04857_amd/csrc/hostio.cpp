// hostio.cpp -- host-only file formats: tuning-cache JSON and checkpoints.
#include "hostio.h"

#include <cctype>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

namespace qhost {

namespace {

// ------------------------------------------------------------ small JSON

struct JVal {
    enum Kind { Null, Bool, Num, Str, Arr, Obj } kind = Null;
    double num = 0.0;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;

    const JVal *get(const char *key) const
    {
        for (const auto &kv : obj)
            if (kv.first == key) return &kv.second;
        return nullptr;
    }
};

struct JParser {
    const std::string &s;
    size_t i = 0;
    std::string err;

    explicit JParser(const std::string &text) : s(text) {}

    void ws()
    {
        while (i < s.size() && std::isspace(static_cast<unsigned char>(s[i]))) i++;
    }
    bool fail(const char *what)
    {
        if (err.empty()) err = std::string(what) + " at offset " + std::to_string(i);
        return false;
    }
    bool lit(const char *w)
    {
        const size_t n = std::strlen(w);
        if (s.compare(i, n, w) != 0) return fail("bad literal");
        i += n;
        return true;
    }
    bool string(std::string *out)
    {
        if (i >= s.size() || s[i] != '"') return fail("expected string");
        i++;
        out->clear();
        while (i < s.size() && s[i] != '"') {
            char c = s[i++];
            if (c == '\\') {
                if (i >= s.size()) return fail("bad escape");
                char e = s[i++];
                switch (e) {
                case 'n': c = '\n'; break;
                case 't': c = '\t'; break;
                case 'r': c = '\r'; break;
                case 'b': c = '\b'; break;
                case 'f': c = '\f'; break;
                case '"': case '\\': case '/': c = e; break;
                default: return fail("unsupported escape");
                }
            }
            out->push_back(c);
        }
        if (i >= s.size()) return fail("unterminated string");
        i++;
        return true;
    }
    bool value(JVal *v, int depth)
    {
        if (depth > 32) return fail("nesting too deep");
        ws();
        if (i >= s.size()) return fail("unexpected end");
        const char c = s[i];
        if (c == '{') {
            v->kind = JVal::Obj;
            i++;
            ws();
            if (i < s.size() && s[i] == '}') {
                i++;
                return true;
            }
            for (;;) {
                ws();
                std::pair<std::string, JVal> kv;
                if (!string(&kv.first)) return false;
                ws();
                if (i >= s.size() || s[i] != ':') return fail("expected ':'");
                i++;
                if (!value(&kv.second, depth + 1)) return false;
                v->obj.push_back(std::move(kv));
                ws();
                if (i < s.size() && s[i] == ',') {
                    i++;
                    continue;
                }
                if (i < s.size() && s[i] == '}') {
                    i++;
                    return true;
                }
                return fail("expected ',' or '}'");
            }
        }
        if (c == '[') {
            v->kind = JVal::Arr;
            i++;
            ws();
            if (i < s.size() && s[i] == ']') {
                i++;
                return true;
            }
            for (;;) {
                JVal e;
                if (!value(&e, depth + 1)) return false;
                v->arr.push_back(std::move(e));
                ws();
                if (i < s.size() && s[i] == ',') {
                    i++;
                    continue;
                }
                if (i < s.size() && s[i] == ']') {
                    i++;
                    return true;
                }
                return fail("expected ',' or ']'");
            }
        }
        if (c == '"') {
            v->kind = JVal::Str;
            return string(&v->str);
        }
        if (c == 't') {
            v->kind = JVal::Bool;
            v->num = 1;
            return lit("true");
        }
        if (c == 'f') {
            v->kind = JVal::Bool;
            return lit("false");
        }
        if (c == 'n') return lit("null");
        const char *b = s.c_str() + i;
        char *e = nullptr;
        v->num = std::strtod(b, &e);
        if (e == b) return fail("bad value");
        v->kind = JVal::Num;
        i += size_t(e - b);
        return true;
    }
    bool parse(JVal *root)
    {
        if (!value(root, 0)) return false;
        ws();
        if (i != s.size()) return fail("trailing characters");
        return true;
    }
};

constexpr const char *kFormat = "qubo-tune-1";

const char *dtype_name(qubo_dtype_t d) { return d == QUBO_FP32 ? "fp32" : "int32"; }

bool int_field(const JVal &o, const char *key, int *out, std::string *msg)
{
    const JVal *v = o.get(key);
    if (!v || v->kind != JVal::Num || v->num != std::floor(v->num) || std::fabs(v->num) > 1e9) {
        *msg = std::string("entry field '") + key + "' missing or not an integer";
        return false;
    }
    *out = int(v->num);
    return true;
}

// Parse a cache text into entries; checks the format tag and device key.
}  // namespace

bool parse_cache(const std::string &text, const std::string &device_key,
                 std::vector<qplan::TuneEntry> *entries, std::string *msg)
{
    JVal root;
    JParser p(text);
    if (!p.parse(&root)) {
        *msg = "tuning cache is not valid JSON: " + p.err;
        return false;
    }
    if (root.kind != JVal::Obj) {
        *msg = "tuning cache must be a JSON object";
        return false;
    }
    const JVal *fmt = root.get("format");
    if (!fmt || fmt->kind != JVal::Str || fmt->str != kFormat) {
        *msg = std::string("tuning cache format must be \"") + kFormat + "\"";
        return false;
    }
    const JVal *dev = root.get("device");
    if (!dev || dev->kind != JVal::Str) {
        *msg = "tuning cache has no device key";
        return false;
    }
    if (dev->str != device_key) {
        *msg = "tuning cache was made on " + dev->str + ", this device is " + device_key;
        return false;
    }
    const JVal *arr = root.get("entries");
    if (!arr || arr->kind != JVal::Arr) {
        *msg = "tuning cache has no entries array";
        return false;
    }
    for (const JVal &o : arr->arr) {
        if (o.kind != JVal::Obj) {
            *msg = "tuning cache entry is not an object";
            return false;
        }
        qplan::TuneEntry e;
        const JVal *dt = o.get("dtype");
        if (!dt || dt->kind != JVal::Str || (dt->str != "int32" && dt->str != "fp32")) {
            *msg = "entry field 'dtype' must be \"int32\" or \"fp32\"";
            return false;
        }
        e.dtype = dt->str == "fp32" ? QUBO_FP32 : QUBO_INT32;
        if (!int_field(o, "n", &e.n, msg) || !int_field(o, "B", &e.B, msg) ||
            !int_field(o, "L", &e.L, msg) || !int_field(o, "tier", &e.tier, msg) ||
            !int_field(o, "vgpr_levels", &e.vgpr_levels, msg))
            return false;
        const JVal *ms = o.get("walk_ms");
        e.walk_ms = (ms && ms->kind == JVal::Num) ? ms->num : 0.0;
        const JVal *sc = o.get("scope");
        if (sc && (sc->kind != JVal::Str || (sc->str != "single" && sc->str != "batch"))) {
            *msg = "entry field 'scope' must be \"single\" or \"batch\"";
            return false;
        }
        e.scope = (sc && sc->str == "batch") ? qplan::kScopeBatch : qplan::kScopeSingle;
        if (!qplan::tune_valid(e, msg)) {
            *msg = "n=" + std::to_string(e.n) + ": " + *msg;
            return false;
        }
        entries->push_back(e);
    }
    return true;
}

std::string format_cache(const std::vector<qplan::TuneEntry> &entries, const std::string &key)
{
    std::ostringstream o;
    o << "{\"format\": \"" << kFormat << "\", \"device\": \"" << key << "\", \"entries\": [";
    for (size_t k = 0; k < entries.size(); k++) {
        const qplan::TuneEntry &e = entries[k];
        char buf[320];
        std::snprintf(buf, sizeof(buf),
                      "%s\n  {\"n\": %d, \"dtype\": \"%s\", \"B\": %d, \"L\": %d, \"tier\": %d, "
                      "\"vgpr_levels\": %d, \"walk_ms\": %.17g, \"scope\": \"%s\"}",
                      k ? "," : "", e.n, dtype_name(e.dtype), e.B, e.L, e.tier, e.vgpr_levels,
                      e.walk_ms, e.scope == qplan::kScopeBatch ? "batch" : "single");
        o << buf;
    }
    o << "\n]}\n";
    return o.str();
}

bool read_file(const char *path, std::string *out, std::string *msg)
{
    std::ifstream f(path, std::ios::binary);
    if (!f) {
        *msg = std::string("cannot open ") + path;
        return false;
    }
    std::ostringstream ss;
    ss << f.rdbuf();
    *out = ss.str();
    if (out->size() > (16u << 20)) {
        *msg = "tuning cache larger than 16 MiB";
        return false;
    }
    return true;
}

bool write_file(const char *path, const std::string &text, std::string *msg)
{
    // write a sibling temporary and rename, so readers never see half a file
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
        if (!f) {
            *msg = std::string("cannot write ") + tmp;
            return false;
        }
        f << text;
        if (!f) {
            *msg = std::string("write failed: ") + tmp;
            return false;
        }
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        *msg = std::string("cannot rename to ") + path;
        return false;
    }
    return true;
}


uint64_t input_hash(const void *Q, int n, qubo_dtype_t dtype)
{
    uint64_t h = 0xcbf29ce484222325ull;
    auto mix = [&h](unsigned char b) {
        h ^= b;
        h *= 0x100000001b3ull;
    };
    const uint32_t head[2] = {uint32_t(n), uint32_t(dtype)};
    for (uint32_t w : head)
        for (int b = 0; b < 4; ++b) mix(static_cast<unsigned char>(w >> (8 * b)));
    const unsigned char *p = static_cast<const unsigned char *>(Q);
    for (size_t i = 0; i < size_t(n) * n * 4; ++i) mix(p[i]);
    return h;
}

namespace {

constexpr const char *kMagic = "qubo-checkpoint 1";



}  // namespace

bool write_ckpt(const char *path, const Ckpt &c, std::string *msg)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) {
        *msg = "cannot write " + tmp + ": " + std::strerror(errno);
        return false;
    }
    int w = std::fprintf(
        f,
        "%s\nn %d\ndtype %d\nqhash %016llx\nplan %d %d %d %d %d\nitems %llu\nnext_item %llu\n"
        "found %d\nenergy_i %lld\nenergy %.17g\nindex %llu\np %d\ntol %.17g\nwalk_ms %.17g\n",
        kMagic, c.n, c.dtype, static_cast<unsigned long long>(c.qhash), c.A, c.B, c.L, c.tier,
        c.vgpr_levels, static_cast<unsigned long long>(c.items),
        static_cast<unsigned long long>(c.next_item), c.found, static_cast<long long>(c.energy_i),
        c.energy, static_cast<unsigned long long>(c.index), c.p, c.tol, c.walk_ms);
    bool ok = w > 0 && std::fflush(f) == 0;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) {
        *msg = "write failed: " + tmp;
        return false;
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        *msg = std::string("cannot rename to ") + path + ": " + std::strerror(errno);
        return false;
    }
    return true;
}

// 1: read; 0: no such file; -1: unreadable or malformed (msg set).
int read_ckpt(const char *path, Ckpt *c, std::string *msg)
{
    FILE *f = std::fopen(path, "r");
    if (!f) {
        if (errno == ENOENT) return 0;
        *msg = std::string("cannot read ") + path + ": " + std::strerror(errno);
        return -1;
    }
    char magic[64] = {0};
    unsigned long long qh = 0, items = 0, next = 0, index = 0;
    long long ei = 0;
    int got = 0;
    bool ok = std::fgets(magic, sizeof magic, f) != nullptr &&
              std::strncmp(magic, kMagic, std::strlen(kMagic)) == 0 &&
              (magic[std::strlen(kMagic)] == '\n' || magic[std::strlen(kMagic)] == 0);
    if (ok) {
        got = std::fscanf(f,
                          " n %d dtype %d qhash %llx plan %d %d %d %d %d items %llu next_item %llu"
                          " found %d energy_i %lld energy %lg index %llu p %d tol %lg walk_ms %lg",
                          &c->n, &c->dtype, &qh, &c->A, &c->B, &c->L, &c->tier, &c->vgpr_levels,
                          &items, &next, &c->found, &ei, &c->energy, &index, &c->p, &c->tol,
                          &c->walk_ms);
        ok = got == 17;
    }
    if (ok) {
        char extra[8];
        ok = std::fscanf(f, " %7s", extra) == EOF;   // nothing may follow
    }
    std::fclose(f);
    c->qhash = qh;
    c->items = items;
    c->next_item = next;
    c->energy_i = ei;
    c->index = index;
    if (ok)
        ok = c->n >= 1 && c->n <= qplan::kMaxN && (c->dtype == QUBO_INT32 || c->dtype == QUBO_FP32) &&
             c->next_item <= c->items && (c->found == 0 || c->found == 1) &&
             (c->found || c->next_item == 0) && c->index < (uint64_t(1) << c->n) &&
             (c->B == 0 || c->A + c->B == c->n) && c->walk_ms >= 0.0;
    if (!ok) {
        *msg = std::string("malformed checkpoint ") + path;
        return -1;
    }
    return 1;
}


}  // namespace qhost
