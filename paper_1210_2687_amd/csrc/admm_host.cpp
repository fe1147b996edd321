// admm_host.cpp — host-only logic of the library (see admm_host.h).
#include "admm_host.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <vector>

namespace admm_host {

namespace {
thread_local std::string g_err;

}  // namespace

admm_status fail(admm_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

const char* last_error() { return g_err.c_str(); }

void prefix_error(const std::string& prefix) { g_err = prefix + g_err; }

bool smooth7(int n) {
    if (n < 1) return false;
    for (int p : {2, 3, 5, 7})
        while (n % p == 0) n /= p;
    return n == 1;
}

admm_status validate(const admm_problem& p) {
    if (p.H < 8 || p.W < 8 || p.H > ADMM_MAX_SIDE || p.W > ADMM_MAX_SIDE)
        return fail(ADMM_E_UNSUPPORTED, "sides %dx%d outside 8..%d", p.H, p.W, ADMM_MAX_SIDE);
    if (!smooth7(p.H) || !smooth7(p.W))
        return fail(ADMM_E_UNSUPPORTED, "sides %dx%d must be 7-smooth (2^a 3^b 5^c 7^d)", p.H, p.W);
    if (!p.kernel || !p.mask) return fail(ADMM_E_INVALID, "null kernel or mask pointer");
    if (p.ksize < 1 || p.ksize % 2 == 0 || p.ksize > std::min(p.H, p.W))
        return fail(ADMM_E_UNSUPPORTED, "kernel side %d must be odd and <= min(H, W)", p.ksize);
    if (p.reg != ADMM_REG_TV && p.reg != ADMM_REG_FRAME && p.reg != ADMM_REG_FRAME_SYNTHESIS)
        return fail(ADMM_E_INVALID, "unknown regulariser %d", p.reg);
    if (p.method != ADMM_METHOD_MD && p.method != ADMM_METHOD_CG) return fail(ADMM_E_INVALID, "unknown method %d", p.method);
    if (p.method == ADMM_METHOD_CG && p.reg == ADMM_REG_FRAME_SYNTHESIS)
        return fail(ADMM_E_UNSUPPORTED, "the synthesis formulation runs with mask decoupling only");
    if (p.reg != ADMM_REG_TV && (p.levels < 1 || p.levels > 4))
        return fail(ADMM_E_UNSUPPORTED, "frame levels %d outside 1..4", p.levels);
    // the kernels address each array with 32-bit byte offsets: the frame's 3J+1
    // coefficient planes (and the TV pair of dual planes) must stay below 4 GiB
    const long long planes = p.reg == ADMM_REG_TV ? 2 : 3LL * p.levels + 1;
    if ((long long)p.H * p.W * planes * (long long)sizeof(float) > 0xFFFFFFFFLL)
        return fail(ADMM_E_UNSUPPORTED, "%dx%d with %lld coefficient planes exceeds 4 GiB per array", p.H, p.W,
                    planes);
    if (!(p.lambda >= 0.0) || !std::isfinite(p.lambda)) return fail(ADMM_E_INVALID, "lambda must be finite and >= 0");
    if (!std::isfinite(p.mu1) || !std::isfinite(p.mu2)) return fail(ADMM_E_INVALID, "mu must be finite");
    double sum = 0.0, asum = 0.0;
    for (int i = 0; i < p.ksize * p.ksize; ++i) {
        if (!std::isfinite(p.kernel[i])) return fail(ADMM_E_INVALID, "non-finite kernel tap %d", i);
        sum += p.kernel[i];
        asum += std::fabs(p.kernel[i]);
    }
    if (asum == 0.0) return fail(ADMM_E_SINGULAR, "kernel is identically zero");
    if (p.reg == ADMM_REG_TV && std::fabs(sum) <= 1e-12 * asum)
        return fail(ADMM_E_SINGULAR, "TV needs a kernel with nonzero sum (DC gain), got %g", sum);
    return ADMM_OK;
}

namespace {

void skip_ws(const char*& p) {
    while (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t') ++p;
}
bool parse_str(const char*& p, std::string& out) {
    skip_ws(p);
    if (*p != '"') return false;
    ++p;
    out.clear();
    while (*p && *p != '"') {
        if (*p == '\\') return false;   // keys and fields never need escapes
        out.push_back(*p++);
    }
    if (*p != '"') return false;
    ++p;
    return true;
}
bool parse_char(const char*& p, char c) {
    skip_ws(p);
    if (*p != c) return false;
    ++p;
    return true;
}

}  // namespace

bool parse_cache(const std::string& text, std::map<std::string, TuneEntry>& out) {
    const char* p = text.c_str();
    if (!parse_char(p, '{')) return false;
    skip_ws(p);
    if (*p == '}') return true;
    for (;;) {
        std::string key;
        if (!parse_str(p, key) || !parse_char(p, ':') || !parse_char(p, '{')) return false;
        TuneEntry e;
        skip_ws(p);
        if (*p != '}') {
            for (;;) {
                std::string f;
                if (!parse_str(p, f) || !parse_char(p, ':')) return false;
                skip_ws(p);
                char* end = nullptr;
                const double v = std::strtod(p, &end);
                if (end == p) return false;
                p = end;
                // tile counts are small non-negative integers and timings finite
                // non-negative numbers: anything else makes the file malformed
                // (and keeps the conversions below defined)
                const bool count = f == "tc" || f == "rows" || f == "rows_512" || f == "rows_1024" || f == "rows_2048" ||
                                   f == "rows_4096" || f == "rows_8192" || f == "rows_16384";
                const bool sched = f == "rsched" || f == "csched";
                if (!std::isfinite(v) || v < 0.0 || (count && (v > kMaxTileCount || v != std::floor(v))) ||
                    (sched && (v >= kScheduleVariants || v != std::floor(v))))
                    return false;
                if (f == "rsched") e.rsched = (int)v;
                else if (f == "csched") e.csched = (int)v;
                if (f == "tc") e.tc = (int)v;
                else if (f == "rows") e.rows = (int)v;
                else if (f == "rows_512") e.rows_c[0] = (int)v;
                else if (f == "rows_1024") e.rows_c[1] = (int)v;
                else if (f == "rows_2048") e.rows_c[2] = (int)v;
                else if (f == "rows_4096") e.rows_c[3] = (int)v;
                else if (f == "rows_8192") e.rows_c[4] = (int)v;
                else if (f == "rows_16384") e.rows_c[5] = (int)v;
                else if (f == "col_us") e.col_us = v;
                else if (f == "row_us") e.row_us = v;
                skip_ws(p);
                if (*p == ',') {
                    ++p;
                    continue;
                }
                break;
            }
        }
        if (!parse_char(p, '}')) return false;
        out[key] = e;
        skip_ws(p);
        if (*p == ',') {
            ++p;
            continue;
        }
        break;
    }
    if (!parse_char(p, '}')) return false;
    skip_ws(p);
    return *p == '\0';   // nothing may follow the object
}

std::string format_cache(const std::map<std::string, TuneEntry>& m) {
    std::string s = "{\n";
    size_t i = 0;
    for (const auto& kv : m) {
        char buf[512];
        std::string extra;
        static const char* names[kRowClasses] = {"rows_512",  "rows_1024", "rows_2048",
                                                 "rows_4096", "rows_8192", "rows_16384"};
        for (int c = 0; c < kRowClasses; ++c)
            if (kv.second.rows_c[c] > 0) extra += ", \"" + std::string(names[c]) + "\": " + std::to_string(kv.second.rows_c[c]);
        if (kv.second.rsched > 0) extra += ", \"rsched\": " + std::to_string(kv.second.rsched);
        if (kv.second.csched > 0) extra += ", \"csched\": " + std::to_string(kv.second.csched);
        std::snprintf(buf, sizeof buf, "{\"tc\": %d, \"rows\": %d%s, \"col_us\": %.3f, \"row_us\": %.3f}",
                      kv.second.tc, kv.second.rows, extra.c_str(), kv.second.col_us, kv.second.row_us);
        s += "  \"" + kv.first + "\": " + buf + (++i < m.size() ? ",\n" : "\n");
    }
    return s + "}\n";
}

// 0: read (or absent: empty map); -1: unreadable or malformed
int read_cache(const char* path, std::map<std::string, TuneEntry>& out) {
    out.clear();
    FILE* f = std::fopen(path, "rb");
    if (!f) return 0;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    std::fclose(f);
    return parse_cache(text, out) ? 0 : -1;
}

int write_cache(const char* path, const std::map<std::string, TuneEntry>& m) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return -1;
    const std::string s = format_cache(m);
    const bool ok = std::fwrite(s.data(), 1, s.size(), f) == s.size();
    if (std::fclose(f) != 0 || !ok) return -1;
    return std::rename(tmp.c_str(), path) == 0 ? 0 : -1;
}

std::string make_key(const admm_problem* probs, int count, const char* arch) {
    std::vector<std::string> sh;
    for (int i = 0; i < count; ++i) {
        char b[48];
        // method CG plans run other kernels: their own entries ("tvcg...", "facg...")
        const char* cg = probs[i].method == ADMM_METHOD_CG ? "cg" : "";
        if (probs[i].reg != ADMM_REG_TV)
            std::snprintf(b, sizeof b, "%s%s%dx%dj%d", probs[i].reg == ADMM_REG_FRAME ? "fa" : "fs", cg,
                          (int)probs[i].H, (int)probs[i].W, (int)probs[i].levels);
        else
            std::snprintf(b, sizeof b, "tv%s%dx%d", cg, (int)probs[i].H, (int)probs[i].W);
        sh.push_back(b);
    }
    std::sort(sh.begin(), sh.end());
    std::string list;
    for (size_t i = 0; i < sh.size();) {
        size_t j = i;
        while (j < sh.size() && sh[j] == sh[i]) ++j;
        if (!list.empty()) list += ",";
        list += sh[i] + "*" + std::to_string(j - i);
        i = j;
    }
    if (list.size() > 160) {   // long ragged batches: a hash of the shape list
        unsigned long long h = 1469598103934665603ull;
        for (unsigned char c : list) h = (h ^ c) * 1099511628211ull;
        char b[40];
        std::snprintf(b, sizeof b, "h%016llx*%d", h, count);
        list = b;
    }
    return std::string(arch) + "|" + list;
}

}  // namespace admm_host

namespace {

int next_smooth7(int n) {
    while (!admm_host::smooth7(n)) ++n;
    return n;
}

}  // namespace

extern "C" admm_status admm_embed_size(int32_t obs_h, int32_t obs_w, int32_t ksize, int32_t* H, int32_t* W) {
    using admm_host::fail;
    if (!H || !W) return fail(ADMM_E_INVALID, "null output pointer");
    if (obs_h < 1 || obs_w < 1 || ksize < 1) return fail(ADMM_E_INVALID, "sizes must be positive");
    if (ksize % 2 == 0) return fail(ADMM_E_UNSUPPORTED, "kernel side %d must be odd", ksize);
    const long long need_h = (long long)obs_h + ksize - 1, need_w = (long long)obs_w + ksize - 1;
    if (need_h > ADMM_MAX_SIDE || need_w > ADMM_MAX_SIDE)
        return fail(ADMM_E_UNSUPPORTED, "unknown domain %lldx%lld above %d", need_h, need_w, ADMM_MAX_SIDE);
    const int h = next_smooth7(std::max<int>(8, (int)need_h)), w = next_smooth7(std::max<int>(8, (int)need_w));
    if (h > ADMM_MAX_SIDE || w > ADMM_MAX_SIDE)
        return fail(ADMM_E_UNSUPPORTED, "no 7-smooth side <= %d holds %lldx%lld", ADMM_MAX_SIDE, need_h, need_w);
    *H = h;
    *W = w;
    return ADMM_OK;
}

extern "C" admm_status admm_embed_observation(const float* y_obs, const uint8_t* obs_mask, int32_t obs_h,
                                              int32_t obs_w, int32_t ksize, int32_t H, int32_t W, float* y,
                                              uint8_t* mask) {
    using admm_host::fail;
    if (!y_obs || !y || !mask) return fail(ADMM_E_INVALID, "null pointer");
    if (obs_h < 1 || obs_w < 1 || ksize < 1 || ksize % 2 == 0) return fail(ADMM_E_INVALID, "bad sizes");
    if ((long long)H < (long long)obs_h + ksize - 1 || (long long)W < (long long)obs_w + ksize - 1)
        return fail(ADMM_E_INVALID, "%dx%d does not hold the unknown domain of a %dx%d observation and a %d kernel", H, W,
                    obs_h, obs_w, ksize);
    const int l = ksize / 2;
    std::fill(y, y + (size_t)H * W, 0.0f);
    std::fill(mask, mask + (size_t)H * W, (uint8_t)0);
    for (int r = 0; r < obs_h; ++r)
        for (int c = 0; c < obs_w; ++c) {
            const size_t s = (size_t)r * obs_w + c, d = (size_t)(r + l) * W + (c + l);
            const uint8_t m = obs_mask ? (obs_mask[s] != 0) : 1;
            mask[d] = m;
            y[d] = m ? y_obs[s] : 0.0f;
        }
    return ADMM_OK;
}
