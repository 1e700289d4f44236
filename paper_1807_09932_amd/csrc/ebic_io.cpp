// ebic_io.cpp -- ingest and export around the evaluation.
//
// Ingest: a delimited text matrix (the EBIC paper, Methods, "Different input
// file formats support": values separated by comma, tab or semicolon; the
// upper-left header cell may be absent) parsed straight into a column-major
// FP32 array that ebic_upload_matrix takes with EBIC_SRC_COL_MAJOR. Lines
// are parsed by several threads; each value is read as a double (correctly
// rounded) and rounded to float, so a value's bits do not depend on the
// thread or the line it is in.
//
// Export: the biclusters of chosen individuals (their columns, and the rows
// of their match masks) as text that R reads with two calls, one per
// dimension (Methods, "Compatibility with R and Bioconductor").
#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ebic.h"
#include "ebic_runtime_internal.h"

namespace {

using ebic::fail;

struct Line {
    const char *b, *e;  // [b, e) without the line break
};

std::vector<Line> split_lines(const std::string &text)
{
    std::vector<Line> out;
    const char *p = text.data(), *end = p + text.size();
    while (p < end) {
        const char *q = static_cast<const char *>(std::memchr(p, '\n', (size_t)(end - p)));
        const char *e = q ? q : end;
        const char *ee = (e > p && e[-1] == '\r') ? e - 1 : e;
        // skip blank lines
        bool blank = true;
        for (const char *t = p; t < ee; ++t)
            if (*t != ' ' && *t != '\t') {
                blank = false;
                break;
            }
        if (!blank) out.push_back({p, ee});
        p = q ? q + 1 : end;
    }
    return out;
}

std::vector<std::string> split_fields(const Line &l, char delim)
{
    std::vector<std::string> f;
    const char *p = l.b;
    while (true) {
        const char *q = p;
        while (q < l.e && *q != delim) ++q;
        std::string s(p, q);
        // trim spaces and surrounding quotes
        size_t a = s.find_first_not_of(' '), z = s.find_last_not_of(' ');
        s = a == std::string::npos ? std::string() : s.substr(a, z - a + 1);
        if (s.size() >= 2 && (s.front() == '"' || s.front() == '\'') && s.back() == s.front())
            s = s.substr(1, s.size() - 2);
        f.push_back(s);
        if (q >= l.e) break;
        p = q + 1;
    }
    return f;
}

bool is_missing_token(const char *b, const char *e)
{
    const size_t n = (size_t)(e - b);
    if (n == 0) return true;
    auto eq = [&](const char *w) { return n == std::strlen(w) && std::strncmp(b, w, n) == 0; };
    return eq("NA") || eq("NaN") || eq("nan") || eq("NAN") || eq("na") || eq("?");
}

// Parse one numeric field [b, e): true on success.
bool parse_value(const char *b, const char *e, float *out)
{
    while (b < e && *b == ' ') ++b;
    while (e > b && e[-1] == ' ') --e;
    if (e - b >= 2 && (*b == '"' || *b == '\'') && e[-1] == *b) {
        ++b;
        --e;
    }
    if (is_missing_token(b, e)) {
        *out = std::nanf("");
        return true;
    }
    char buf[64];
    const size_t n = (size_t)(e - b);
    if (n >= sizeof(buf)) return false;
    std::memcpy(buf, b, n);
    buf[n] = 0;
    char *stop = nullptr;
    errno = 0;
    const double v = std::strtod(buf, &stop);
    if (stop == buf || *stop != 0) return false;
    *out = (float)v;
    return true;
}

bool numeric(const std::string &s)
{
    float v;
    return parse_value(s.data(), s.data() + s.size(), &v) && !is_missing_token(s.data(), s.data() + s.size());
}

char detect_delimiter(const Line &l)
{
    const char cands[3] = {'\t', ';', ','};
    char best = ',';
    size_t best_n = 0;
    for (char c : cands) {
        const size_t n = (size_t)std::count(l.b, l.e, c);
        if (n > best_n) {
            best_n = n;
            best = c;
        }
    }
    return best;
}

char *dup_string(const std::string &s)
{
    char *p = static_cast<char *>(std::malloc(s.size() + 1));
    if (!p) throw std::bad_alloc();
    std::memcpy(p, s.c_str(), s.size() + 1);
    return p;
}

}  // namespace

using namespace ebic;

extern "C" {

ebic_status ebic_free_text_matrix(ebic_text_matrix *m)
{
    if (!m) return EBIC_OK;
    std::free(m->values);
    if (m->row_names) {
        for (int64_t r = 0; r < m->rows; ++r) std::free(m->row_names[r]);
        std::free(m->row_names);
    }
    if (m->col_names) {
        for (int32_t c = 0; c < m->cols; ++c) std::free(m->col_names[c]);
        std::free(m->col_names);
    }
    std::memset(m, 0, sizeof(*m));
    return EBIC_OK;
}

ebic_status ebic_read_delimited(const char *path, char delimiter, int32_t header, int32_t row_names,
                                int32_t threads, ebic_text_matrix *out)
{
    ebic_text_matrix m{};
    const ebic_status st = guarded([&] {
        if (!path || !out) fail(EBIC_EINVAL, "path and out are required");
        std::memset(out, 0, sizeof(*out));
        if (!(delimiter == 0 || delimiter == ',' || delimiter == '\t' || delimiter == ';'))
            fail(EBIC_EINVAL, "delimiter must be 0 (detect), ',', '\\t' or ';'");
        FILE *f = std::fopen(path, "rb");
        if (!f) fail(EBIC_ENOENT, std::string("cannot open ") + path);
        std::string text;
        {
            std::fseek(f, 0, SEEK_END);
            const long sz = std::ftell(f);
            std::fseek(f, 0, SEEK_SET);
            text.resize(sz > 0 ? (size_t)sz : 0);
            const size_t got = text.empty() ? 0 : std::fread(&text[0], 1, text.size(), f);
            std::fclose(f);
            if (got != text.size()) fail(EBIC_EINVAL, std::string("short read of ") + path);
        }
        const std::vector<Line> lines = split_lines(text);
        if (lines.empty()) fail(EBIC_EINVAL, "no data lines");
        const char d = delimiter ? delimiter : detect_delimiter(lines[0]);
        const std::vector<std::string> first = split_fields(lines[0], d);
        const std::vector<std::string> second =
            lines.size() > 1 ? split_fields(lines[1], d) : std::vector<std::string>();
        // A header row has a non-numeric field past the first one (or a first
        // field that is not a number while the next line's is).
        bool hdr;
        if (header >= 0) hdr = header != 0;
        else {
            hdr = false;
            for (size_t j = 1; j < first.size(); ++j)
                if (!first[j].empty() && !numeric(first[j]) && !is_missing_token(first[j].data(), first[j].data() + first[j].size()))
                    hdr = true;
        }
        const std::vector<std::string> &probe = hdr ? second : first;
        if (hdr && lines.size() < 2) fail(EBIC_EINVAL, "a header but no data line");
        bool names;
        if (row_names >= 0) names = row_names != 0;
        else names = !probe.empty() && !numeric(probe[0]) &&
                     !is_missing_token(probe[0].data(), probe[0].data() + probe[0].size());
        const int64_t ncols = (int64_t)probe.size() - (names ? 1 : 0);
        if (ncols < 1) fail(EBIC_EINVAL, "no value columns");
        const int64_t nrows = (int64_t)lines.size() - (hdr ? 1 : 0);
        m.rows = nrows;
        m.cols = (int32_t)ncols;
        m.delimiter = d;
        m.values = static_cast<float *>(std::malloc(sizeof(float) * (size_t)nrows * (size_t)ncols));
        if (!m.values) throw std::bad_alloc();
        if (hdr) {
            // The header names the value columns; with row names it may or
            // may not carry the upper-left cell.
            const size_t skip = first.size() == (size_t)ncols + 1 ? 1 : 0;
            if (first.size() - skip != (size_t)ncols)
                fail(EBIC_EINVAL, "header has " + std::to_string(first.size()) + " fields for " +
                                      std::to_string(ncols) + " columns");
            m.col_names = static_cast<char **>(std::calloc((size_t)ncols, sizeof(char *)));
            if (!m.col_names) throw std::bad_alloc();
            for (int64_t c = 0; c < ncols; ++c) m.col_names[c] = dup_string(first[skip + (size_t)c]);
        }
        if (names) {
            m.row_names = static_cast<char **>(std::calloc((size_t)nrows, sizeof(char *)));
            if (!m.row_names) throw std::bad_alloc();
        }
        // Parse the data lines in parallel.
        const int nt = std::max(1, std::min<int>(threads > 0 ? threads : 1, 64));
        std::vector<std::string> errors((size_t)nt);
        auto work = [&](int t) {
            const int64_t r0 = nrows * t / nt, r1 = nrows * (t + 1) / nt;
            for (int64_t r = r0; r < r1 && errors[t].empty(); ++r) {
                const Line &l = lines[(size_t)r + (hdr ? 1 : 0)];
                const char *p = l.b;
                int64_t c = names ? -1 : 0;
                while (true) {
                    const char *q = p;
                    while (q < l.e && *q != d) ++q;
                    if (c == -1) {
                        std::string s(p, q);
                        size_t a = s.find_first_not_of(' '), z = s.find_last_not_of(' ');
                        s = a == std::string::npos ? std::string() : s.substr(a, z - a + 1);
                        if (s.size() >= 2 && (s.front() == '"' || s.front() == '\'') && s.back() == s.front())
                            s = s.substr(1, s.size() - 2);
                        m.row_names[r] = dup_string(s);
                    } else if (c < ncols) {
                        float v;
                        if (!parse_value(p, q, &v)) {
                            errors[t] = "line " + std::to_string(r + (hdr ? 2 : 1)) + ", field " +
                                        std::to_string(c + (names ? 2 : 1)) + ": not a number";
                            break;
                        }
                        m.values[(size_t)c * (size_t)nrows + (size_t)r] = v;
                    }
                    ++c;
                    if (q >= l.e) break;
                    p = q + 1;
                }
                if (errors[t].empty() && c != ncols)
                    errors[t] = "line " + std::to_string(r + (hdr ? 2 : 1)) + " has " +
                                std::to_string(c + (names ? 1 : 0)) + " fields, expected " +
                                std::to_string(ncols + (names ? 1 : 0));
            }
        };
        std::vector<std::thread> pool;
        for (int t = 1; t < nt; ++t) pool.emplace_back(work, t);
        work(0);
        for (auto &th : pool) th.join();
        for (auto &e : errors)
            if (!e.empty()) fail(EBIC_EINVAL, e);
        *out = m;
    });
    if (st != EBIC_OK) ebic_free_text_matrix(&m);
    return st;
}

ebic_status ebic_write_biclusters(const char *path, int64_t rows, int32_t n_ind, const int32_t *offsets,
                                  const int32_t *cols, const uint64_t *matched_mask, int32_t n_out,
                                  const int32_t *which, const char *const *row_names,
                                  const char *const *col_names)
{
    return guarded([&] {
        if (!path || n_out < 0 || (n_out > 0 && (!which || !offsets || !cols || !matched_mask)))
            fail(EBIC_EINVAL, "bad arguments");
        for (int32_t b = 0; b < n_out; ++b)
            if (which[b] < 0 || which[b] >= n_ind) fail(EBIC_EINVAL, "individual index out of range");
        if (rows < 1) fail(EBIC_EINVAL, "rows must be >= 1");
        const int64_t words = (rows + 63) / 64;
        FILE *f = std::fopen(path, "wb");
        if (!f) fail(EBIC_ENOENT, std::string("cannot create ") + path);
        std::string buf;
        auto flush = [&] {
            if (!buf.empty() && std::fwrite(buf.data(), 1, buf.size(), f) != buf.size()) {
                std::fclose(f);
                fail(EBIC_EINVAL, std::string("write failed: ") + path);
            }
            buf.clear();
        };
        buf += "# EBIC biclusters: " + std::to_string(n_out) + "\n";
        for (int32_t b = 0; b < n_out; ++b) {
            const int32_t i = which[b];
            const uint64_t *mask = matched_mask + (size_t)i * (size_t)words;
            int64_t nr = 0;
            for (int64_t w = 0; w < words; ++w) nr += __builtin_popcountll(mask[w]);
            const int32_t k = offsets[i + 1] - offsets[i];
            buf += "bicluster\t" + std::to_string(b + 1) + "\t" + std::to_string(nr) + "\t" + std::to_string(k) + "\n";
            buf += "rows";
            for (int64_t w = 0; w < words; ++w) {
                uint64_t x = mask[w];
                while (x) {
                    const int bit = __builtin_ctzll(x);
                    x &= x - 1;
                    const int64_t r = w * 64 + bit;
                    buf += '\t';
                    buf += row_names ? std::string(row_names[r]) : std::to_string(r + 1);
                }
                if (buf.size() > (1 << 20)) flush();
            }
            buf += "\ncols";
            for (int32_t j = offsets[i]; j < offsets[i + 1]; ++j) {
                buf += '\t';
                buf += col_names ? std::string(col_names[cols[j]]) : std::to_string(cols[j] + 1);
            }
            buf += '\n';
        }
        flush();
        if (std::fclose(f) != 0) fail(EBIC_EINVAL, std::string("close failed: ") + path);
    });
}

}  // extern "C"
