// autotune.hip -- the autotuner of the batched form.
//
// For every row length the given items transform, it times candidate radix
// orders (partitions of the power-of-two part into radices 16/8/4/2 with at
// most one pass more than the fewest, each in a few orders, together with the
// 3s and 5s) and two choices of rows per work-group on the generic row kernel;
// for every (u size, v size) pair of their transposes it times tile shapes
// TU x TV (x G slices), and the same radix orders in the FFT step fused with
// that transpose (the unit the batched form runs by default: its best radix
// order differs from the separate row kernel's).  Timing uses HIP events on a private stream over a
// synthetic array of about 16 M complex values.  The winners are written to a
// small JSON cache tagged with the device architecture and library version;
// plans built with that cache (fft_batch_plan's tune_cache) use them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/fftrw.h"
#include "decomp.hpp"
#include "errors.hpp"
#include "kernels.hpp"
#include "tune.hpp"

namespace fftrw {

hipError_t launch_twiddles(void *out, int64_t n, bool fp64, hipStream_t s);
hipError_t launch_fft_rows(const FftDesc &d, bool fp64, int dir, const void *in, void *out, double scale,
                           hipStream_t s);
hipError_t launch_xpose(const XposeDesc &d, size_t esz, const void *in, void *out, hipStream_t s);
hipError_t launch_fft_xpose_generic(const FftDesc &f, const XposeDesc &d, bool fp64, int dir, const void *in,
                                    void *out, double scale, hipStream_t s);
int factor_radices(int64_t n, int *rad);

std::string tune_device_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    return std::string(prop.gcnArchName);
}

namespace {

std::string json_string(const std::string &txt, const std::string &key)
{
    const std::string k = "\"" + key + "\"";
    size_t p = txt.find(k);
    if (p == std::string::npos) return "";
    p = txt.find('"', txt.find(':', p + k.size()) + 1);
    if (p == std::string::npos) return "";
    const size_t e = txt.find('"', p + 1);
    return e == std::string::npos ? "" : txt.substr(p + 1, e - p - 1);
}

// integers of one field inside an object: "key": 12 or "key": [8, 8, 3]
std::vector<long long> json_ints(const std::string &obj, const std::string &key)
{
    std::vector<long long> out;
    const std::string k = "\"" + key + "\"";
    size_t p = obj.find(k);
    if (p == std::string::npos) return out;
    p = obj.find(':', p + k.size());
    if (p == std::string::npos) return out;
    ++p;
    while (p < obj.size() && (obj[p] == ' ' || obj[p] == '\t')) ++p;
    const bool list = p < obj.size() && obj[p] == '[';
    const size_t end = list ? obj.find(']', p) : obj.find_first_of(",}", p);
    std::string body = obj.substr(list ? p + 1 : p, (end == std::string::npos ? obj.size() : end) - (list ? p + 1 : p));
    std::replace(body.begin(), body.end(), ',', ' ');
    std::istringstream is(body);
    long long v;
    while (is >> v) out.push_back(v);
    return out;
}

std::vector<std::string> json_objects(const std::string &txt, const std::string &array_key)
{
    std::vector<std::string> out;
    size_t p = txt.find("\"" + array_key + "\"");
    if (p == std::string::npos) return out;
    p = txt.find('[', p);
    if (p == std::string::npos) return out;
    int depth = 0;
    size_t start = 0;
    for (size_t i = p + 1; i < txt.size(); ++i) {
        if (txt[i] == '{') {
            if (depth++ == 0) start = i;
        } else if (txt[i] == '}') {
            if (--depth == 0) out.push_back(txt.substr(start, i - start + 1));
        } else if (txt[i] == ']' && depth == 0) {
            break;
        }
    }
    return out;
}

void factor235(int n, int *e2, int *e3, int *e5)
{
    *e2 = *e3 = *e5 = 0;
    while (n % 2 == 0) n /= 2, ++*e2;
    while (n % 3 == 0) n /= 3, ++*e3;
    while (n % 5 == 0) n /= 5, ++*e5;
}

void partitions(int left, int maxpart, std::vector<int> &cur, std::vector<std::vector<int>> &out)
{
    if (left == 0) {
        out.push_back(cur);
        return;
    }
    for (int p = std::min(left, maxpart); p >= 1; --p) {
        cur.push_back(p);
        partitions(left - p, p, cur, out);
        cur.pop_back();
    }
}

std::vector<std::vector<int>> row_candidates(int N)
{
    int e2, e3, e5;
    factor235(N, &e2, &e3, &e5);
    std::vector<std::vector<int>> parts;
    std::vector<int> cur;
    partitions(e2, 4, cur, parts);
    size_t fewest = 100;
    for (auto &p : parts) fewest = std::min(fewest, p.size());
    std::set<std::vector<int>> seen;
    std::vector<std::vector<int>> out;
    for (auto &p : parts) {
        if (p.size() > fewest + 1) continue;
        std::vector<int> two;
        for (int x : p) two.push_back(1 << x);
        std::vector<int> odd;
        for (int i = 0; i < e3; ++i) odd.push_back(3);
        for (int i = 0; i < e5; ++i) odd.push_back(5);
        std::vector<int> a = two, b;
        a.insert(a.end(), odd.begin(), odd.end());           // powers of two first
        b = odd;
        b.insert(b.end(), two.begin(), two.end());           // 3s and 5s first
        std::vector<int> c(a.rbegin(), a.rend());             // reversed
        for (auto &v : {a, b, c})
            if (seen.insert(v).second) out.push_back(v);
    }
    return out;
}

struct Timer {
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool ok = true;
    Timer()
    {
        ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
             hipEventCreate(&e1) == hipSuccess;
    }
    ~Timer()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
    }
    template <class F> float time(F &&launch, int reps)
    {
        for (int i = 0; i < 2; ++i)
            if (launch() != hipSuccess) return -1.f;
        if (hipEventRecord(e0, s) != hipSuccess) return -1.f;
        for (int i = 0; i < reps; ++i)
            if (launch() != hipSuccess) return -1.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.f;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.f;
        return ms / reps;
    }
};

int64_t pow2ceil64(int64_t x)
{
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

bool tune_load(const std::string &path, const std::string &device, const std::string &version, TuneTable *out)
{
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string txt = ss.str();
    TuneTable t;
    t.device = json_string(txt, "device");
    t.version = json_string(txt, "version");
    if (t.device != device || t.version != version) return false;
    for (const std::string &o : json_objects(txt, "rows")) {
        auto n = json_ints(o, "n"), rw = json_ints(o, "rows_per_wg"), rad = json_ints(o, "radix");
        if (n.size() != 1 || rw.size() != 1 || rad.empty()) continue;
        RowTune r;
        r.rows_per_wg = (int)rw[0];
        for (long long x : rad) r.radix.push_back((int)x);
        t.rows[(int)n[0]] = r;
    }
    for (const std::string &o : json_objects(txt, "tiles")) {
        auto nu = json_ints(o, "nu"), nv = json_ints(o, "nv"), tu = json_ints(o, "tu"), tv = json_ints(o, "tv"),
             g = json_ints(o, "g");
        if (nu.size() != 1 || nv.size() != 1 || tu.size() != 1 || tv.size() != 1 || g.size() != 1) continue;
        t.tiles[{(int)nu[0], (int)nv[0]}] = TileTune{(int)tu[0], (int)tv[0], (int)g[0]};
    }
    for (const std::string &o : json_objects(txt, "fused")) {
        auto n = json_ints(o, "n"), nv = json_ints(o, "nv"), rad = json_ints(o, "radix");
        if (n.size() != 1 || nv.size() != 1 || rad.empty()) continue;
        std::vector<int> r;
        for (long long x : rad) r.push_back((int)x);
        t.fused[{(int)n[0], (int)nv[0]}] = r;
    }
    *out = t;
    return true;
}

bool tune_save(const std::string &path, const TuneTable &t)
{
    std::ofstream f(path);
    if (!f) return false;
    f << "{\n  \"device\": \"" << t.device << "\",\n  \"version\": \"" << t.version << "\",\n  \"rows\": [";
    bool first = true;
    for (const auto &kv : t.rows) {
        f << (first ? "\n" : ",\n") << "    {\"n\": " << kv.first << ", \"rows_per_wg\": " << kv.second.rows_per_wg
          << ", \"radix\": [";
        for (size_t i = 0; i < kv.second.radix.size(); ++i) f << (i ? ", " : "") << kv.second.radix[i];
        f << "]}";
        first = false;
    }
    f << "\n  ],\n  \"tiles\": [";
    first = true;
    for (const auto &kv : t.tiles) {
        f << (first ? "\n" : ",\n") << "    {\"nu\": " << kv.first.first << ", \"nv\": " << kv.first.second
          << ", \"tu\": " << kv.second.TU << ", \"tv\": " << kv.second.TV << ", \"g\": " << kv.second.G << "}";
        first = false;
    }
    f << "\n  ],\n  \"fused\": [";
    first = true;
    for (const auto &kv : t.fused) {
        f << (first ? "\n" : ",\n") << "    {\"n\": " << kv.first.first << ", \"nv\": " << kv.first.second
          << ", \"radix\": [";
        for (size_t i = 0; i < kv.second.size(); ++i) f << (i ? ", " : "") << kv.second[i];
        f << "]}";
        first = false;
    }
    f << "\n  ]\n}\n";
    return (bool)f;
}

}  // namespace fftrw

using namespace fftrw;

extern "C" int fft_autotune(int n, const fft_item_desc *items, const char *cache_path, unsigned flags)
{
    g_last_error.clear();
    (void)flags;
    if (n < 1 || !items || !cache_path) return fail(FFTRW_E_ARG, "null items or cache path, or n < 1");
    // row lengths and transpose (u, v) pairs of every item's pipeline
    std::set<int> lengths;
    std::set<std::pair<int, int>> pairs;
    for (int i = 0; i < n; ++i) {
        const fft_item_desc &it = items[i];
        if (it.M < 2 || it.M > kMaxDims) return fail(FFTRW_E_SIZE, "items have M = 2..5");
        Status st = check_dims(it.M, it.dims);
        if (!st) return fail(st);
        std::vector<int8_t> order(it.M * it.M);
        if (it.has_order) {
            std::memcpy(order.data(), it.order, order.size());
        } else {
            int rc = fft_order_search(it.M, it.dims, it.P, FFTRW_OWN_LITERAL, nullptr, nullptr, nullptr, nullptr,
                                      nullptr, nullptr, order.data(), nullptr);
            if (rc) return rc;
        }
        for (int t = 0; t < it.M; ++t) {
            const int u = order[t * it.M + it.M - 1];
            const int v = t + 1 < it.M ? order[(t + 1) * it.M + it.M - 1] : it.M - 1;
            lengths.insert((int)it.dims[u]);
            pairs.insert({(int)it.dims[u], (int)it.dims[v]});
        }
    }
    TuneTable table;
    table.device = tune_device_name();
    table.version = fft_version();
    const int64_t cap = 1 << 24;  // complex values per timing array
    void *a = nullptr, *b = nullptr, *tw = nullptr;
    if (hipMalloc(&a, cap * 8) != hipSuccess || hipMalloc(&b, cap * 8) != hipSuccess ||
        hipMalloc(&tw, 4096 * 8) != hipSuccess) {
        (void)hipGetLastError();
        if (a) (void)hipFree(a);
        if (b) (void)hipFree(b);
        return fail(FFTRW_E_NOMEM, "autotuner buffers");
    }
    if (hipMemset(a, 0, cap * 8) != hipSuccess) return fail(FFTRW_E_DEVICE, "autotuner buffer clear");
    Timer tm;
    int rc = tm.ok ? FFTRW_OK : fail(FFTRW_E_DEVICE, "autotuner stream/events");
    for (int N : lengths) {
        if (rc) break;
        if (N > 4096) continue;
        if (launch_twiddles(tw, N, false, tm.s) != hipSuccess) {
            rc = fail(FFTRW_E_DEVICE, "autotuner twiddles");
            break;
        }
        int64_t rw0 = 1;
        while (rw0 * 2 <= 256 && rw0 * 2 * N <= 4096) rw0 *= 2;
        float best = -1.f;
        RowTune win;
        for (const std::vector<int> &rad : row_candidates(N)) {
            for (int64_t rw : {rw0, rw0 / 2}) {
                if (rw < 1) continue;
                FftDesc d;
                std::memset(&d, 0, sizeof(d));
                d.N = N;
                d.npass = (int)rad.size();
                for (size_t q = 0; q < rad.size(); ++q) d.radix[q] = rad[q];
                d.rows_per_wg = (int)rw;
                d.lanes_per_row = (int)(256 / rw);
                d.nrows = cap / N;
                d.tw = tw;
                const float ms = tm.time([&] { return launch_fft_rows(d, false, -1, a, b, 1.0, tm.s); }, 5);
                if (ms > 0.f && (best < 0.f || ms < best)) {
                    best = ms;
                    win.rows_per_wg = (int)rw;
                    win.radix = rad;
                }
            }
        }
        if (best > 0.f) table.rows[N] = win;
    }
    for (const auto &pr : pairs) {
        if (rc) break;
        const int Nu = pr.first, Nv = pr.second;
        float best = -1.f;
        TileTune win;
        const int64_t S = std::max<int64_t>(1, cap / ((int64_t)Nu * Nv));
        for (auto tt : std::vector<std::pair<int, int>>{{64, 64}, {32, 32}, {16, 16}, {64, 16}, {16, 64}, {32, 64},
                                                        {64, 32}, {8, 64}, {64, 8}}) {
            const int TU = (int)std::min<int64_t>(tt.first, pow2ceil64(Nu));
            const int TV = (int)std::min<int64_t>(tt.second, pow2ceil64(Nv));
            const int64_t G = std::min<int64_t>(std::min<int64_t>(256, S), std::max<int64_t>(1, 4096 / (TU * TV)));
            XposeDesc d;
            std::memset(&d, 0, sizeof(d));
            d.Nu = Nu;
            d.Nv = Nv;
            d.a_sv = Nu;   // A = [slice][v][u]
            d.b_su = Nv;   // B = [slice][u][v]
            d.nbat = 1;
            d.bsize[0] = S;
            d.ba[0] = d.bb[0] = (int64_t)Nu * Nv;
            d.nslices = S;
            d.TU = TU;
            d.TV = TV;
            d.G = (int)G;
            d.tiles_u = (Nu + TU - 1) / TU;
            d.tiles_v = (Nv + TV - 1) / TV;
            d.tiles_g = (S + G - 1) / G;
            const float ms = tm.time([&] { return launch_xpose(d, 8, a, b, tm.s); }, 5);
            if (ms > 0.f && (best < 0.f || ms < best)) {
                best = ms;
                win = TileTune{TU, TV, (int)G};
            }
        }
        if (best > 0.f) table.tiles[pr] = win;
        // the FFT step along u fused with this transpose, per radix order
        if (Nu + 1 > 4096) continue;
        if (launch_twiddles(tw, Nu, false, tm.s) != hipSuccess) {
            rc = fail(FFTRW_E_DEVICE, "autotuner twiddles");
            break;
        }
        XposeDesc x;
        std::memset(&x, 0, sizeof(x));
        x.Nu = Nu;
        x.Nv = Nv;
        x.a_sv = Nu;
        x.b_su = Nv;
        x.nbat = 1;
        x.bsize[0] = S;
        x.ba[0] = x.bb[0] = (int64_t)Nu * Nv;
        x.nslices = S;
        // the built-in order first; another wins only by a clear margin (3%),
        // since the times of near-equal orders differ by noise on this array
        int def[kMaxPasses];
        const int ndef = factor_radices(Nu, def);
        std::vector<std::vector<int>> cands{std::vector<int>(def, def + ndef)};
        for (const std::vector<int> &rad : row_candidates(Nu))
            if (rad != cands[0]) cands.push_back(rad);
        float fdef = -1.f, fbest = -1.f;
        std::vector<int> fwin;
        for (const std::vector<int> &rad : cands) {
            FftDesc f;
            std::memset(&f, 0, sizeof(f));
            f.N = Nu;
            f.npass = (int)rad.size();
            for (size_t q = 0; q < rad.size(); ++q) f.radix[q] = rad[q];
            f.nrows = S * Nv;
            f.tw = tw;
            const float ms = tm.time([&] { return launch_fft_xpose_generic(f, x, false, -1, a, b, 1.0, tm.s); }, 10);
            if (ms <= 0.f) continue;
            if (fdef < 0.f) {
                fdef = fbest = ms;
                fwin = rad;
            } else if (ms < fbest && ms < 0.97f * fdef) {
                fbest = ms;
                fwin = rad;
            }
        }
        if (fbest > 0.f) table.fused[pr] = fwin;
    }
    (void)hipFree(a);
    (void)hipFree(b);
    (void)hipFree(tw);
    if (rc) return rc;
    if (!tune_save(cache_path, table)) return fail(FFTRW_E_ARG, std::string("cannot write ") + cache_path);
    return FFTRW_OK;
}
