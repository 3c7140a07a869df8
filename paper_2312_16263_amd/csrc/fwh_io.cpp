// Host-side ingestion of the OpenCFD-FWH file layout (Appendix A of the paper):
// the control file (a Fortran namelist), the surface geometry file, the
// observer file and the per-step FW-H dataset files, read into the flat,
// time-major arrays the C ABI of include/fwh.h takes.  Plain C++17, no device
// code; the frame files are read by a pool of std::threads (one frame per
// task) straight into the caller's arrays.
//
// Layouts (Appendix A2 and Sec. III A as described in the text; the dataset
// layout of Appendix A3 is a reading, its figure being unavailable):
//  * FWH_Surface_Geo.dat (ASCII): a text line ("variables=x,y,z,n1,n2,n3,dS"),
//    the number of Faces, then per Face a line "nx ny nz" (one of them 1)
//    followed by nx*ny*nz lines "x y z n1 n2 n3 dS".  Panels are numbered in
//    file order over all Faces.
//  * observers.dat (ASCII): one observer per line, "x y z".
//  * control.fwh: Fortran namelist groups "&name key = value, ... /" with "!"
//    comments; keys are returned lower-case with their value text.
//  * FWH-xxxxxxxx.dat, xxxxxxxx the zero-padded iteration step: per Face the
//    block dimensions then, per subface in the geometry file's order, the
//    density, the three velocity components and the pressure pulsation.
//    ASCII (format 1): a line "nx ny nz" then one line "rho u v w p'" per
//    subface.  Binary (format 0): Fortran unformatted sequential records, each
//    framed by its 4-byte length: per Face a record of three int32 dimensions
//    and a record of 5*nx*ny*nz float64 values, variable-major (all rho, then
//    u, v, w, p').
#include "../../include/fwh_io.h"

#include <algorithm>
#include <atomic>
#include <cctype>
#include <cerrno>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

namespace {

thread_local std::string g_io_error;

int io_fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_io_error = buf;
    return code;
}

bool read_file(const char *path, std::string &out) {
    FILE *f = fopen(path, "rb");
    if (!f) return false;
    std::string s;
    char buf[1 << 16];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
    fclose(f);
    out.swap(s);
    return true;
}

// Whitespace/comma-separated numeric tokens; Fortran 'd'/'D' exponents accepted.
struct Tok {
    const char *p, *e;
    int line = 1;
    explicit Tok(const std::string &s) : p(s.data()), e(s.data() + s.size()) {}
    void skip_sep() {
        while (p < e && (isspace((unsigned char)*p) || *p == ',')) {
            if (*p == '\n') ++line;
            ++p;
        }
    }
    void skip_line() {
        while (p < e && *p != '\n') ++p;
        if (p < e) {
            ++p;
            ++line;
        }
    }
    bool number(double &v) {
        skip_sep();
        if (p >= e) return false;
        char buf[64];
        int n = 0;
        while (p + n < e && n < 63 && !isspace((unsigned char)p[n]) && p[n] != ',') {
            char c = p[n];
            buf[n] = (c == 'd' || c == 'D') ? 'e' : c;
            ++n;
        }
        if (n == 63 && p + n < e && !isspace((unsigned char)p[n]) && p[n] != ',') return false;
        buf[n] = 0;
        char *end = nullptr;
        errno = 0;
        v = strtod(buf, &end);
        if (end != buf + n || n == 0) return false;
        if (errno == ERANGE && (v == HUGE_VAL || v == -HUGE_VAL)) return false;  // overflow; underflow is kept
        p += n;
        return true;
    }
    bool integer(int64_t &v) {
        double d;
        if (!number(d) || !(d > -9.0e15 && d < 9.0e15)) return false;
        v = (int64_t)d;
        return (double)v == d;
    }
};

std::string lower(std::string s) {
    for (auto &c : s) c = (char)tolower((unsigned char)c);
    return s;
}

}  // namespace

extern "C" {

const char *fwh_io_last_error(void) { return g_io_error.c_str(); }

int fwh_io_geometry_read(const char *path, int64_t *n_faces, int64_t *n_panels, int64_t *face_dims, double *y,
                         double *normal, double *dS, int64_t cap_faces, int64_t cap_panels) {
    g_io_error.clear();
    if (!path || !n_faces || !n_panels) return io_fail(FWH_IO_EINVAL, "fwh_io_geometry_read: null argument");
    std::string s;
    if (!read_file(path, s)) return io_fail(FWH_IO_EFILE, "cannot read %s", path);
    Tok t(s);
    t.skip_line();  // "variables=..."
    int64_t nf;
    if (!t.integer(nf) || nf < 1) return io_fail(FWH_IO_EFORMAT, "%s: bad Face count on line %d", path, t.line);
    const bool fill = y && normal && dS;
    int64_t np = 0;
    for (int64_t f = 0; f < nf; ++f) {
        int64_t d[3];
        for (int i = 0; i < 3; ++i)
            if (!t.integer(d[i]) || d[i] < 1)
                return io_fail(FWH_IO_EFORMAT, "%s: bad dimensions of Face %lld near line %d", path, (long long)f,
                               t.line);
        if (face_dims && f < cap_faces)
            for (int i = 0; i < 3; ++i) face_dims[3 * f + i] = d[i];
        const int64_t n = d[0] * d[1] * d[2];
        for (int64_t q = 0; q < n; ++q, ++np) {
            double v[7];
            for (int i = 0; i < 7; ++i)
                if (!t.number(v[i]))
                    return io_fail(FWH_IO_EFORMAT, "%s: bad subface record %lld of Face %lld near line %d", path,
                                   (long long)q, (long long)f, t.line);
            if (fill) {
                if (np >= cap_panels) return io_fail(FWH_IO_ESIZE, "%s: more than %lld panels", path, (long long)cap_panels);
                for (int i = 0; i < 3; ++i) {
                    y[3 * np + i] = v[i];
                    normal[3 * np + i] = v[3 + i];
                }
                dS[np] = v[6];
            }
        }
    }
    *n_faces = nf;
    *n_panels = np;
    return FWH_IO_OK;
}

int fwh_io_observers_read(const char *path, int64_t *n_obs, double *x_obs, int64_t cap) {
    g_io_error.clear();
    if (!path || !n_obs) return io_fail(FWH_IO_EINVAL, "fwh_io_observers_read: null argument");
    std::string s;
    if (!read_file(path, s)) return io_fail(FWH_IO_EFILE, "cannot read %s", path);
    int64_t n = 0;
    size_t pos = 0;
    int line = 0;
    while (pos < s.size()) {
        size_t nl = s.find('\n', pos);
        if (nl == std::string::npos) nl = s.size();
        std::string ln = s.substr(pos, nl - pos);
        pos = nl + 1;
        ++line;
        bool blank = true;
        for (char c : ln) blank = blank && isspace((unsigned char)c);
        if (blank) continue;
        Tok t(ln);
        double v[3];
        for (int i = 0; i < 3; ++i)
            if (!t.number(v[i])) return io_fail(FWH_IO_EFORMAT, "%s: line %d is not 'x y z'", path, line);
        if (x_obs) {
            if (n >= cap) return io_fail(FWH_IO_ESIZE, "%s: more than %lld observers", path, (long long)cap);
            for (int i = 0; i < 3; ++i) x_obs[3 * n + i] = v[i];
        }
        ++n;
    }
    *n_obs = n;
    return FWH_IO_OK;
}

int fwh_io_control_read(const char *path, fwh_io_kv *kv, int32_t cap, int32_t *n) {
    g_io_error.clear();
    if (!path || !n) return io_fail(FWH_IO_EINVAL, "fwh_io_control_read: null argument");
    std::string s;
    if (!read_file(path, s)) return io_fail(FWH_IO_EFILE, "cannot read %s", path);
    // strip comments (outside quotes)
    std::string body;
    bool inq = false;
    char q = 0;
    for (size_t i = 0; i < s.size(); ++i) {
        const char c = s[i];
        if (inq) {
            body += c;
            if (c == q) inq = false;
        } else if (c == '\'' || c == '"') {
            inq = true;
            q = c;
            body += c;
        } else if (c == '!') {
            while (i < s.size() && s[i] != '\n') ++i;
            body += '\n';
        } else {
            body += c;
        }
    }
    int32_t count = 0;
    size_t i = 0;
    std::string group;
    while (i < body.size()) {
        const char c = body[i];
        if (c == '&' || c == '$') {  // group start
            size_t j = i + 1;
            while (j < body.size() && (isalnum((unsigned char)body[j]) || body[j] == '_')) ++j;
            group = lower(body.substr(i + 1, j - i - 1));
            if (group == "end") group.clear();  // the older "&end" terminator
            i = j;
            continue;
        }
        if (c == '/') {  // group end
            group.clear();
            ++i;
            continue;
        }
        if (isalpha((unsigned char)c) && !group.empty()) {
            size_t j = i;
            while (j < body.size() && (isalnum((unsigned char)body[j]) || body[j] == '_' || body[j] == '%')) ++j;
            std::string key = lower(body.substr(i, j - i));
            size_t k = j;
            while (k < body.size() && isspace((unsigned char)body[k])) ++k;
            if (k >= body.size() || body[k] != '=')
                return io_fail(FWH_IO_EFORMAT, "%s: expected '=' after '%s'", path, key.c_str());
            ++k;
            while (k < body.size() && isspace((unsigned char)body[k])) ++k;
            // the value runs to the group's end or to the next "name =" (so an array
            // value "1, 2, 3" stays whole); quoted text may hold any of these
            std::string val;
            size_t m = k;
            size_t keep = 0;  // characters up to the end of the last quoted run are kept
            while (m < body.size()) {
                const char ch = body[m];
                if (ch == '\'' || ch == '"') {  // quoted text is copied as written
                    size_t e = m + 1;
                    for (;;) {
                        const size_t f = body.find(ch, e);
                        if (f == std::string::npos) return io_fail(FWH_IO_EFORMAT, "%s: unterminated string", path);
                        if (f + 1 < body.size() && body[f + 1] == ch) {  // a doubled quote stands for one
                            e = f + 2;
                            continue;
                        }
                        e = f + 1;
                        break;
                    }
                    val.append(body, m, e - m);
                    keep = val.size();
                    m = e;
                    continue;
                }
                if (ch == '/' || ch == '&' || ch == '$') break;  // group end, next group
                if (isalpha((unsigned char)ch) && m > k &&
                    (isspace((unsigned char)body[m - 1]) || body[m - 1] == ',')) {
                    size_t e = m;
                    while (e < body.size() && (isalnum((unsigned char)body[e]) || body[e] == '_' || body[e] == '%')) ++e;
                    while (e < body.size() && isspace((unsigned char)body[e])) ++e;
                    if (e < body.size() && body[e] == '=') break;
                }
                val += ch;
                ++m;
            }
            k = m;
            while (val.size() > keep && (isspace((unsigned char)val.back()) || val.back() == ',')) val.pop_back();
            if (key.size() >= sizeof(fwh_io_kv::key) || val.size() >= sizeof(fwh_io_kv::value) ||
                group.size() >= sizeof(fwh_io_kv::group))
                return io_fail(FWH_IO_ESIZE, "%s: entry '%s' longer than an fwh_io_kv field", path, key.c_str());
            if (kv) {
                if (count >= cap) return io_fail(FWH_IO_ESIZE, "%s: more than %d entries", path, (int)cap);
                snprintf(kv[count].key, sizeof kv[count].key, "%s", key.c_str());
                snprintf(kv[count].value, sizeof kv[count].value, "%s", val.c_str());
                snprintf(kv[count].group, sizeof kv[count].group, "%s", group.c_str());
            }
            ++count;
            i = k;
            continue;
        }
        ++i;
    }
    *n = count;
    return FWH_IO_OK;
}

}  // extern "C"

namespace {

// One frame file into time-major row n of rho [N][P], u [3][N][P], pp [N][P];
// the file's Faces must be those of dims [F][3].
template <typename T>
int read_frame(const char *path, int format, int64_t F, const int64_t *dims, int64_t P, int64_t N, int64_t n, T *rho,
               T *u, T *pp, std::string &err) {
    std::string s;
    if (!read_file(path, s)) {
        err = std::string("cannot read ") + path;
        return FWH_IO_EFILE;
    }
    const int64_t NP = N * P;
    T *dst[5] = {rho + n * P, u + n * P, u + NP + n * P, u + 2 * NP + n * P, pp + n * P};
    auto bad = [&](int64_t f, const char *what) {
        err = std::string(path) + ": Face " + std::to_string(f) + ": " + what;
        return FWH_IO_EFORMAT;
    };
    int64_t pnl = 0;
    if (format == FWH_IO_ASCII) {
        Tok t(s);
        for (int64_t f = 0; f < F; ++f) {
            for (int i = 0; i < 3; ++i) {
                int64_t d;
                if (!t.integer(d)) return bad(f, "missing dimensions");
                if (d != dims[3 * f + i]) return bad(f, "dimensions differ from the geometry file");
            }
            const int64_t m = dims[3 * f] * dims[3 * f + 1] * dims[3 * f + 2];
            for (int64_t q = 0; q < m; ++q, ++pnl) {
                for (int v = 0; v < 5; ++v) {
                    double x;
                    if (!t.number(x)) return bad(f, "missing or bad value");
                    dst[v][pnl] = (T)x;
                }
            }
        }
        double extra;
        if (t.number(extra)) return bad(F, "values past the last Face");
        return FWH_IO_OK;
    }
    // binary: Fortran unformatted sequential records [uint32 len][data][uint32 len]
    size_t off = 0;
    auto record = [&](const char *&data, uint32_t want) -> bool {
        uint32_t len, tail;
        if (off + 8 + (size_t)want > s.size()) return false;
        memcpy(&len, s.data() + off, 4);
        if (len != want) return false;
        memcpy(&tail, s.data() + off + 4 + len, 4);
        if (tail != len) return false;
        data = s.data() + off + 4;
        off += 8 + (size_t)len;
        return true;
    };
    for (int64_t f = 0; f < F; ++f) {
        const char *data;
        if (!record(data, 12)) return bad(f, "bad dimension record");
        int32_t d[3];
        memcpy(d, data, 12);
        for (int i = 0; i < 3; ++i)
            if (d[i] != dims[3 * f + i]) return bad(f, "dimensions differ from the geometry file");
        const int64_t m = dims[3 * f] * dims[3 * f + 1] * dims[3 * f + 2];
        if (5 * m * 8 > (int64_t)UINT32_MAX) return bad(f, "Face too large for one record");
        if (!record(data, (uint32_t)(5 * m * 8))) return bad(f, "bad value record");
        for (int v = 0; v < 5; ++v) {
            const char *src = data + (size_t)v * m * 8;
            if constexpr (sizeof(T) == 8) {
                memcpy(dst[v] + pnl, src, (size_t)m * 8);
            } else {
                for (int64_t q = 0; q < m; ++q) {
                    double x;
                    memcpy(&x, src + q * 8, 8);
                    dst[v][pnl + q] = (T)x;
                }
            }
        }
        pnl += m;
    }
    if (off != s.size()) return bad(F, "bytes past the last Face");
    return FWH_IO_OK;
}

bool face_panels(int64_t F, const int64_t *dims, int64_t &P) {
    P = 0;
    for (int64_t f = 0; f < F; ++f) {
        for (int i = 0; i < 3; ++i)
            if (dims[3 * f + i] < 1 || dims[3 * f + i] > INT32_MAX) return false;
        P += dims[3 * f] * dims[3 * f + 1] * dims[3 * f + 2];
    }
    return F >= 1;
}

}  // namespace

extern "C" {

int fwh_io_frame_path(const char *dir, int64_t step, char *out, int64_t cap) {
    g_io_error.clear();
    if (!dir || !out || cap < 1) return io_fail(FWH_IO_EINVAL, "fwh_io_frame_path: null argument");
    if (step < 0 || step > 99999999) return io_fail(FWH_IO_EINVAL, "fwh_io_frame_path: step %lld outside 8 digits", (long long)step);
    const int n = snprintf(out, (size_t)cap, "%s/FWH-%08lld.dat", dir, (long long)step);
    if (n < 0 || n >= cap) return io_fail(FWH_IO_ESIZE, "fwh_io_frame_path: buffer too small");
    return FWH_IO_OK;
}

int fwh_io_frames_read(const char *dir, int64_t kstep_start, int64_t delta_step, int64_t n_frames, int32_t format,
                       int64_t n_faces, const int64_t *face_dims, int32_t out_dtype, void *rho, void *u, void *pp,
                       int32_t n_threads) {
    g_io_error.clear();
    if (!dir || !face_dims || !rho || !u || !pp) return io_fail(FWH_IO_EINVAL, "fwh_io_frames_read: null argument");
    if (n_frames < 1 || delta_step < 1 || kstep_start < 0 || kstep_start + (n_frames - 1) * delta_step > 99999999)
        return io_fail(FWH_IO_EINVAL, "fwh_io_frames_read: need n_frames, delta_step >= 1 and steps within 8 digits");
    if (format != FWH_IO_BINARY && format != FWH_IO_ASCII)
        return io_fail(FWH_IO_EINVAL, "fwh_io_frames_read: bad format %d", (int)format);
    if (out_dtype != 0 && out_dtype != 1) return io_fail(FWH_IO_EINVAL, "fwh_io_frames_read: bad out_dtype %d", (int)out_dtype);
    int64_t P;
    if (!face_panels(n_faces, face_dims, P)) return io_fail(FWH_IO_EINVAL, "fwh_io_frames_read: bad Face dimensions");
    int nt = n_threads > 0 ? n_threads : (int)std::max(1u, std::thread::hardware_concurrency());
    nt = (int)std::min<int64_t>(nt, n_frames);
    std::atomic<int64_t> next(0);
    std::atomic<bool> failed(false);
    std::vector<std::string> errs(nt);
    std::vector<int> codes(nt, FWH_IO_OK);
    std::vector<int64_t> at(nt, -1);
    auto worker = [&](int w) {
        char path[4096];
        for (;;) {
            if (failed.load()) return;
            const int64_t n = next.fetch_add(1);
            if (n >= n_frames) return;
            snprintf(path, sizeof path, "%s/FWH-%08lld.dat", dir, (long long)(kstep_start + n * delta_step));
            const int st = out_dtype == 0
                               ? read_frame<double>(path, format, n_faces, face_dims, P, n_frames, n,
                                                    static_cast<double *>(rho), static_cast<double *>(u),
                                                    static_cast<double *>(pp), errs[w])
                               : read_frame<float>(path, format, n_faces, face_dims, P, n_frames, n,
                                                   static_cast<float *>(rho), static_cast<float *>(u),
                                                   static_cast<float *>(pp), errs[w]);
            if (st != FWH_IO_OK) {
                codes[w] = st;
                at[w] = n;
                failed.store(true);
                return;
            }
        }
    };
    std::vector<std::thread> pool;
    for (int w = 1; w < nt; ++w) pool.emplace_back(worker, w);
    worker(0);
    for (auto &th : pool) th.join();
    if (failed.load()) {  // report the earliest failing frame among those read
        int best = -1;
        for (int w = 0; w < nt; ++w)
            if (codes[w] != FWH_IO_OK && (best < 0 || at[w] < at[best])) best = w;
        return io_fail(codes[best], "%s", errs[best].c_str());
    }
    return FWH_IO_OK;
}

int fwh_io_frame_write(const char *path, int32_t format, int64_t n_faces, const int64_t *face_dims,
                       const double *rho, const double *u1, const double *u2, const double *u3, const double *pp) {
    g_io_error.clear();
    if (!path || !face_dims || !rho || !u1 || !u2 || !u3 || !pp)
        return io_fail(FWH_IO_EINVAL, "fwh_io_frame_write: null argument");
    if (format != FWH_IO_BINARY && format != FWH_IO_ASCII)
        return io_fail(FWH_IO_EINVAL, "fwh_io_frame_write: bad format %d", (int)format);
    int64_t P;
    if (!face_panels(n_faces, face_dims, P)) return io_fail(FWH_IO_EINVAL, "fwh_io_frame_write: bad Face dimensions");
    FILE *f = fopen(path, format == FWH_IO_ASCII ? "w" : "wb");
    if (!f) return io_fail(FWH_IO_EFILE, "cannot write %s", path);
    const double *src[5] = {rho, u1, u2, u3, pp};
    int64_t pnl = 0;
    for (int64_t fc = 0; fc < n_faces; ++fc) {
        const int64_t *d = face_dims + 3 * fc;
        const int64_t m = d[0] * d[1] * d[2];
        if (format == FWH_IO_ASCII) {
            fprintf(f, "%lld %lld %lld\n", (long long)d[0], (long long)d[1], (long long)d[2]);
            for (int64_t q = 0; q < m; ++q) {
                const int64_t i = pnl + q;
                fprintf(f, "%.17g %.17g %.17g %.17g %.17g\n", rho[i], u1[i], u2[i], u3[i], pp[i]);
            }
        } else {
            if (5 * m * 8 > (int64_t)UINT32_MAX) {
                fclose(f);
                return io_fail(FWH_IO_ESIZE, "fwh_io_frame_write: Face %lld too large for one record", (long long)fc);
            }
            const int32_t dd[3] = {(int32_t)d[0], (int32_t)d[1], (int32_t)d[2]};
            uint32_t len = 12;
            fwrite(&len, 4, 1, f);
            fwrite(dd, 4, 3, f);
            fwrite(&len, 4, 1, f);
            len = (uint32_t)(5 * m * 8);
            fwrite(&len, 4, 1, f);
            for (int v = 0; v < 5; ++v) fwrite(src[v] + pnl, 8, (size_t)m, f);
            fwrite(&len, 4, 1, f);
        }
        pnl += m;
    }
    const bool bad = ferror(f) != 0;
    if (fclose(f) != 0 || bad) return io_fail(FWH_IO_EFILE, "write error on %s", path);
    return FWH_IO_OK;
}

int fwh_io_geometry_write(const char *path, int64_t n_faces, const int64_t *face_dims, const double *y,
                          const double *normal, const double *dS) {
    g_io_error.clear();
    if (!path || !face_dims || !y || !normal || !dS) return io_fail(FWH_IO_EINVAL, "fwh_io_geometry_write: null argument");
    int64_t P;
    if (!face_panels(n_faces, face_dims, P)) return io_fail(FWH_IO_EINVAL, "fwh_io_geometry_write: bad Face dimensions");
    FILE *f = fopen(path, "w");
    if (!f) return io_fail(FWH_IO_EFILE, "cannot write %s", path);
    fprintf(f, "variables=x,y,z,n1,n2,n3,dS\n%lld\n", (long long)n_faces);
    int64_t pnl = 0;
    for (int64_t fc = 0; fc < n_faces; ++fc) {
        const int64_t *d = face_dims + 3 * fc;
        fprintf(f, "%lld %lld %lld\n", (long long)d[0], (long long)d[1], (long long)d[2]);
        for (int64_t q = 0; q < d[0] * d[1] * d[2]; ++q, ++pnl)
            fprintf(f, "%.17g %.17g %.17g %.17g %.17g %.17g %.17g\n", y[3 * pnl], y[3 * pnl + 1], y[3 * pnl + 2],
                    normal[3 * pnl], normal[3 * pnl + 1], normal[3 * pnl + 2], dS[pnl]);
    }
    const bool bad = ferror(f) != 0;
    if (fclose(f) != 0 || bad) return io_fail(FWH_IO_EFILE, "write error on %s", path);
    return FWH_IO_OK;
}

}  // extern "C"
