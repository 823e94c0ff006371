// The tuned table: per (type, batch form, op pair, size) kernel choice and
// launch shape, measured by the autotuner (paper_1304_7053_amd/tune.py) and
// stored as versioned JSON.  Loaded once per process from SBG_TUNE_FILE, else
// from tuned.json next to this library; an empty SBG_TUNE_FILE, a missing
// file or a version other than 1 leaves the table empty (built-in rules).
//
// The reader accepts the subset of JSON the tuner writes: a top-level object
// whose "version" is a number and whose "entries" is an array of flat
// objects with string and number values; every other member is skipped.
#include <dlfcn.h>

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>

#include "sbg_internal.h"

namespace sbg {
namespace {

constexpr int kVersion = 1;
constexpr int kMaxDepth = 64;

struct Table {
    bool loaded = false;
    std::string path;
    int version = 0;
    int count = 0;
    TunedEntry e[4][2][2][2][17];   // type, pointer form, a_trans, b_trans, size
    bool has[4][2][2][2][17];
};

class Reader {
public:
    explicit Reader(const std::string& t) : s_(t) {}
    bool ok() const { return ok_; }
    void ws()
    {
        while (i_ < s_.size() && std::isspace((unsigned char)s_[i_])) ++i_;
    }
    bool eat(char c)
    {
        ws();
        if (i_ < s_.size() && s_[i_] == c) {
            ++i_;
            return true;
        }
        return false;
    }
    char peek()
    {
        ws();
        return i_ < s_.size() ? s_[i_] : '\0';
    }
    std::string str()
    {
        std::string out;
        if (!eat('"')) return fail(), out;
        while (i_ < s_.size() && s_[i_] != '"') {
            if (s_[i_] == '\\' && i_ + 1 < s_.size()) ++i_;
            out += s_[i_++];
        }
        if (i_ >= s_.size()) return fail(), out;
        ++i_;
        return out;
    }
    double num()
    {
        ws();
        const char* b = s_.c_str() + i_;
        char* e = nullptr;
        const double v = std::strtod(b, &e);
        if (e == b) return fail(), 0.0;
        i_ += (size_t)(e - b);
        return v;
    }
    // an integer field: 0 unless the number is finite and fits an int (a
    // double outside int's range must not be converted)
    int integer()
    {
        const double v = num();
        return (v >= -2147483648.0 && v <= 2147483647.0) ? (int)v : 0;
    }
    // skip any value (nesting deeper than kMaxDepth fails the read instead of
    // recursing without bound)
    void skip(int depth = 0)
    {
        if (depth > kMaxDepth) return fail();
        const char c = peek();
        if (c == '"') {
            str();
        } else if (c == '{') {
            eat('{');
            if (eat('}')) return;
            do {
                str();
                if (!eat(':')) return fail();
                skip(depth + 1);
            } while (ok_ && eat(','));
            if (!eat('}')) fail();
        } else if (c == '[') {
            eat('[');
            if (eat(']')) return;
            do skip(depth + 1);
            while (ok_ && eat(','));
            if (!eat(']')) fail();
        } else if (c == 't' || c == 'f' || c == 'n') {
            while (i_ < s_.size() && std::isalpha((unsigned char)s_[i_])) ++i_;
        } else {
            num();
        }
    }
    void fail() { ok_ = false; }

private:
    const std::string& s_;
    size_t i_ = 0;
    bool ok_ = true;
};

int path_code(const std::string& p)
{
    if (p == "mfma") return 1;
    if (p == "team") return 2;
    if (p == "staged") return 3;
    return 0;
}

// One entry object; adds it to the table when its key fields are valid.
void read_entry(Reader& r, Table& t)
{
    std::string type, form, ops, path;
    int size = 0, unroll = 0, wg = 0, xcd = 0;
    if (!r.eat('{')) return r.fail();
    if (!r.eat('}')) {
        do {
            const std::string key = r.str();
            if (!r.eat(':')) return r.fail();
            if (r.peek() == '"') {
                const std::string v = r.str();
                if (key == "type") type = v;
                else if (key == "form") form = v;
                else if (key == "ops") ops = v;
                else if (key == "path") path = v;
            } else if (r.peek() == '-' || std::isdigit((unsigned char)r.peek())) {
                const int v = r.integer();
                if (key == "size") size = v;
                else if (key == "unroll") unroll = v;
                else if (key == "wg_per_cu") wg = v;
                else if (key == "xcd_chunk") xcd = v;
            } else {
                r.skip();
            }
        } while (r.ok() && r.eat(','));
        if (!r.eat('}')) return r.fail();
    }
    const int ti = type == "s" ? 0 : type == "d" ? 1 : type == "c" ? 2 : type == "z" ? 3 : -1;
    const int fi = form == "strided" ? 0 : form == "pointer" ? 1 : -1;
    if (ti < 0 || fi < 0 || ops.size() != 2 || size < 1 || size > 16) return;
    const auto tr = [](char c) { return c == 'T' || c == 't' || c == 'C' || c == 'c'; };
    const int at = tr(ops[0]) ? 1 : 0, bt = tr(ops[1]) ? 1 : 0;
    TunedEntry& e = t.e[ti][fi][at][bt][size];
    e.path = path_code(path);
    e.unroll = unroll >= 0 && unroll <= 8 ? unroll : 0;
    e.wg_per_cu = wg >= 0 && wg <= 32 ? wg : 0;
    e.xcd_chunk = xcd >= 0 && xcd <= (1 << 20) ? xcd : 0;
    t.has[ti][fi][at][bt][size] = true;
    ++t.count;
}

void parse(const std::string& text, Table& t)
{
    Reader r(text);
    if (!r.eat('{')) return;
    int version = 0;
    Table tmp;
    std::memset(tmp.has, 0, sizeof(tmp.has));
    if (!r.eat('}')) {
        do {
            const std::string key = r.str();
            if (!r.eat(':')) return;
            if (key == "version") {
                version = r.integer();
            } else if (key == "entries") {
                if (!r.eat('[')) return;
                if (!r.eat(']')) {
                    do read_entry(r, tmp);
                    while (r.ok() && r.eat(','));
                    if (!r.eat(']')) return;
                }
            } else {
                r.skip();
            }
        } while (r.ok() && r.eat(','));
    }
    if (!r.ok() || version != kVersion) return;
    std::memcpy(t.e, tmp.e, sizeof(t.e));
    std::memcpy(t.has, tmp.has, sizeof(t.has));
    t.count = tmp.count;
    t.version = version;
}

std::string default_path()
{
    Dl_info info;
    if (dladdr(reinterpret_cast<void*>(&tuned_entry), &info) && info.dli_fname) {
        std::string p(info.dli_fname);
        const size_t slash = p.rfind('/');
        return (slash == std::string::npos ? std::string(".") : p.substr(0, slash)) + "/tuned.json";
    }
    return "tuned.json";
}

Table& table()
{
    static Table t;
    static std::once_flag once;
    std::call_once(once, [] {
        std::memset(t.has, 0, sizeof(t.has));
        const char* env = std::getenv("SBG_TUNE_FILE");
        t.path = env ? std::string(env) : default_path();
        t.loaded = true;
        if (t.path.empty()) return;
        std::ifstream f(t.path);
        if (!f) return;
        std::stringstream ss;
        ss << f.rdbuf();
        parse(ss.str(), t);
    });
    return t;
}

}  // namespace

const TunedEntry* tuned_entry(int type, bool pointer_form, bool a_trans, bool b_trans, int size)
{
    if (type < 0 || type > 3 || size < 1 || size > 16) return nullptr;
    const Table& t = table();
    const int f = pointer_form ? 1 : 0, at = a_trans ? 1 : 0, bt = b_trans ? 1 : 0;
    return t.has[type][f][at][bt][size] ? &t.e[type][f][at][bt][size] : nullptr;
}

int tuned_table_info(char* buf, int len)
{
    if (!buf || len <= 0) return -1;
    const Table& t = table();
    const int w = std::snprintf(buf, (size_t)len, "file=%s version=%d entries=%d", t.path.c_str(), t.version, t.count);
    return w < 0 ? -1 : t.count;
}

}  // namespace sbg
