// fdwave autotuner: times the tile variants, axis-0 chunk lengths and shot-group
// sizes of the step launches on scratch fields of a grid and remembers the fastest
// launch shapes per (GPU architecture, HIP runtime, problem class), optionally in a
// JSON-lines cache file.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fdw_host.h"

namespace fdh {

// ---------------------------------------------------------------------------
// autotuner: remembered launch shapes per (arch, runtime, problem class)
// ---------------------------------------------------------------------------

struct Tuned {
    int variant = 1, chunk = 0, group = 1;
    int variant_plain = 0, chunk_plain = 0;   // launches without accumulator access (0: same)
    double ms = 0.0;
};

std::mutex g_tune_mu;
std::map<std::string, Tuned> g_tuned;
bool g_tune_loaded = false;

std::string device_tag()
{
    int dev = 0, rt = 0;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    (void)hipRuntimeGetVersion(&rt);
    return arch + "|hip" + std::to_string(rt);
}

std::string tune_key(const Geo& G, int nshot)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s|%dd|o%d|%s|acc%s|%dx%dx%d|s%d", device_tag().c_str(), G.ndim,
             2 * G.r, G.dtype == FD_F64 ? "f64" : "f32", G.acc_dtype == FD_F64 ? "f64" : "f32",
             G.n0, G.n1, G.n2, nshot);
    return buf;
}

const char* tune_file() { return std::getenv("FDWAVE_TUNE_CACHE"); }

// Reads "key" and the numbers after "variant", "chunk", "max_group", "variant_plain",
// "chunk_plain" and "ms" from one JSON line written by tune_save (no general JSON parser
// is needed for that format).
bool parse_line(const std::string& ln, std::string* key, Tuned* t)
{
    auto str_after = [&](const char* name, std::string* out) {
        const std::string pat = std::string("\"") + name + "\": \"";
        size_t p = ln.find(pat);
        if (p == std::string::npos) return false;
        p += pat.size();
        size_t q = ln.find('"', p);
        if (q == std::string::npos) return false;
        *out = ln.substr(p, q - p);
        return true;
    };
    auto num_after = [&](const char* name, double* out) {
        const std::string pat = std::string("\"") + name + "\": ";
        size_t p = ln.find(pat);
        if (p == std::string::npos) return false;
        *out = std::atof(ln.c_str() + p + pat.size());
        return true;
    };
    double v, c, g, ms, vp = 0.0, cp = 0.0;
    if (!str_after("key", key) || !num_after("variant", &v) || !num_after("chunk", &c) ||
        !num_after("max_group", &g) || !num_after("ms", &ms))
        return false;
    (void)num_after("variant_plain", &vp);   // absent in entries with one launch shape
    (void)num_after("chunk_plain", &cp);
    t->variant = (int)v;
    t->chunk = (int)c;
    t->group = (int)g;
    t->variant_plain = (int)vp;
    t->chunk_plain = (int)cp;
    t->ms = ms;
    return true;
}

void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = tune_file();
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        std::string key;
        Tuned t;
        if (parse_line(line, &key, &t)) g_tuned[key] = t;   // later lines win
    }
    std::fclose(f);
}

void tune_save_locked(const std::string& key, const Tuned& t)
{
    g_tuned[key] = t;
    const char* path = tune_file();
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f,
                 "{\"key\": \"%s\", \"variant\": %d, \"chunk\": %d, \"max_group\": %d, "
                 "\"variant_plain\": %d, \"chunk_plain\": %d, \"ms\": %.6f}\n",
                 key.c_str(), t.variant, t.chunk, t.group, t.variant_plain, t.chunk_plain, t.ms);
    std::fclose(f);
}

// Applies the remembered launch shape of (G, nshot), if any; returns whether there was one.
bool apply_tuned(Geo& G, int nshot)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tuned.find(tune_key(G, nshot));
    if (it == g_tuned.end()) return false;
    const fdw::Variant v = fdw::variant_shape(G.ndim, it->second.variant);
    if (v.tz == 0 || G.n2 % v.vz != 0) return false;
    G.variant = it->second.variant;
    if (G.chunk == 0) G.chunk = it->second.chunk;
    if (G.max_group == 0) G.max_group = it->second.group;
    if (G.variant_plain == 0) {
        G.variant_plain = it->second.variant_plain;
        if (G.chunk_plain == 0) G.chunk_plain = it->second.chunk_plain;
    }
    return true;
}

int autotune(const fd_grid* grid, int nshot, const fd_opts* opts, int steps, fd_opts* best,
             double* best_ms, hipStream_t s)
{
    Geo G;
    int rc = check_grid(grid, opts, &G);
    if (rc) return rc;
    if (!best) return fail(FD_E_ARG, "best is null");
    if (steps < 1) return fail(FD_E_ARG, "steps must be >= 1");
    // small grids give launches of tens of microseconds: time more of them
    steps *= (int)std::max<int64_t>(1, std::min<int64_t>(64, ((int64_t)1 << 26) / std::max<int64_t>(G.ncell, 1)));
    nshot = std::max(nshot, 1);
    // candidate shapes: variants that fit, shot groups, chunk lengths
    std::vector<int> groups = {1};
    if (nshot >= 2) groups.push_back(2);
    if (nshot >= 4) groups.push_back(4);
    int gmax = 1;
    for (int g : groups) gmax = std::max(gmax, g);
    struct Scoped {
        std::vector<void*> p;
        ~Scoped() { for (void* q : p) (void)hipFree(q); }
    } mem;
    // time the row layout the sweeps run: rows padded to 64 elements when the
    // contiguous extent needs it (the key stays the caller's extents)
    pad_rows(&G);
    const size_t es = dsize(G.dtype);
    const size_t np = (size_t)G.ncell_pad;
    void *c = nullptr, *ua = nullptr, *ub = nullptr, *acc = nullptr;
    HIPCHK(hipMalloc(&c, np * es)); mem.p.push_back(c);
    HIPCHK(hipMalloc(&ua, np * es * gmax)); mem.p.push_back(ua);
    HIPCHK(hipMalloc(&ub, np * es * gmax)); mem.p.push_back(ub);
    HIPCHK(hipMalloc(&acc, np * dsize(G.acc_dtype))); mem.p.push_back(acc);
    HIPCHK(hipMemsetAsync(c, 0, np * es, s));
    HIPCHK(hipMemsetAsync(ua, 0, np * es * gmax, s));
    HIPCHK(hipMemsetAsync(ub, 0, np * es * gmax, s));
    HIPCHK(hipMemsetAsync(acc, 0, np * dsize(G.acc_dtype), s));
    // the typical accumulating launch of a sweep adds to the f32 partial sums, when
    // the sweeps keep them
    void* part = nullptr;
    if (use_partials(G)) {
        HIPCHK(hipMalloc(&part, np * sizeof(float))); mem.p.push_back(part);
        HIPCHK(hipMemsetAsync(part, 0, np * sizeof(float), s));
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    struct Ev { hipEvent_t a, b; ~Ev() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } evs{e0, e1};
    // per shot-group size: the fastest shape of the launches that add kernel terms and,
    // separately, of the launches that touch no accumulator (the sweeps alternate them)
    struct Best { double ms = 1e300; int variant = 0, chunk = 0; };
    std::map<int, Best> best_acc, best_plain, best_same;
    auto time_launches = [&](const Geo& T, const Plan& P, const Group& gr, fdw::StepArgs a, int terms,
                             double* ms_out) -> int {
        void *prev = ua, *cur = ub;
        for (int n = 0; n < steps + 1; ++n) {   // one untimed warm-up launch
            if (n == 1) HIPCHK(hipEventRecord(e0, s));
            a.ucur = cur;
            a.unew = prev;
            set_acc(a, terms, 1);
            a.part = terms ? part : nullptr;
            a.part_mode = part && terms ? fdw::PM_ADD : fdw::PM_DIRECT;
            int rc2 = step_group(T, P, gr, a, s);
            if (rc2) return rc2;
            std::swap(prev, cur);
        }
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        *ms_out = ms / steps;
        return FD_OK;
    };
    for (int variant = 1; variant <= fdw::variant_count(G.ndim); ++variant) {
        const fdw::Variant v = fdw::variant_shape(G.ndim, variant);
        if (G.n2 % v.vz != 0) continue;
        // 2D rows of four cells per lane time well in isolation but ran real 2048^2
        // sweeps at 120 against 208 Gcell-updates/s for two cells per lane: not a 2D
        // candidate
        if (G.ndim == 2 && v.vz == 4) continue;
        std::vector<int> chunks = {0, G.n0, G.n0 / 2, G.n0 / 4, G.n0 / 8, 256, 128, 64};
        // 2D marches serialise their rows: short chunks keep the most blocks in flight
        if (G.ndim == 2) chunks.insert(chunks.end(), {2, 4, 8});
        std::sort(chunks.begin(), chunks.end());
        chunks.erase(std::unique(chunks.begin(), chunks.end()), chunks.end());
        for (int group : groups) {
            if (group > v.max_shots) continue;
            for (int chunk : chunks) {
                if (chunk != 0 && (chunk < (G.ndim == 2 ? 2 : 2 * G.r) || chunk > G.n0)) continue;
                Geo T = G;
                T.variant = variant;
                T.auto_variant = false;
                T.chunk = chunk;
                T.max_group = group;
                T.variant_plain = 0;
                T.timing = nullptr;
                Scratch sc(s);
                Plan P;
                if ((rc = make_plan(T, nullptr, false, s, sc, &P))) return rc;
                Group gr = P.groups[0];
                gr.size = group;
                fdw::StepArgs a = base_args(T, P, c, 0.1);
                a.acc = acc;
                double ms_acc = 0.0, ms_plain = 0.0;
                if ((rc = time_launches(T, P, gr, a, 3, &ms_acc))) return rc;
                if ((rc = time_launches(T, P, gr, a, 0, &ms_plain))) return rc;
                const int resolved = chunk == 0 ? P.chunk : chunk;
                Best& ba = best_acc[group];
                if (ms_acc < ba.ms) ba = Best{ms_acc, variant, resolved};
                Best& bp = best_plain[group];
                if (ms_plain < bp.ms) bp = Best{ms_plain, variant, resolved};
                Best& bs = best_same[group];
                if (ms_acc + ms_plain < bs.ms) bs = Best{ms_acc + ms_plain, variant, resolved};
            }
        }
    }
    Tuned bestv;
    double best_per_shot = 1e300;
    for (int group : groups) {
        if (!best_acc.count(group) || !best_plain.count(group)) continue;
        // 2D: one shape for both launch kinds.  Separately timed shapes mispredict 2D
        // sweeps (small grids whose launches share cache-resident data): real sweeps
        // with a second shape for the plain launches ran up to 30% slower than with
        // the accumulating launches' own shape.
        const Best& ba = G.ndim == 3 ? best_acc[group] : best_same[group];
        const Best& bp = G.ndim == 3 ? best_plain[group] : best_same[group];
        const double per_pair = G.ndim == 3 ? ba.ms + bp.ms : ba.ms;
        if (per_pair / group < best_per_shot) {
            best_per_shot = per_pair / group;
            bestv.variant = ba.variant;
            bestv.chunk = ba.chunk;
            bestv.group = group;
            bestv.variant_plain = bp.variant;
            bestv.chunk_plain = bp.chunk;
            bestv.ms = per_pair / 2;
        }
    }
    HIPCHK(hipStreamSynchronize(s));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        tune_save_locked(tune_key(G, nshot), bestv);
    }
    if (opts) *best = *opts;
    else std::memset(best, 0, sizeof(*best));
    best->variant = bestv.variant;
    best->chunk = bestv.chunk;
    best->max_group = bestv.group;
    best->variant_plain = bestv.variant_plain;
    best->chunk_plain = bestv.chunk_plain;
    if (best_ms) *best_ms = bestv.ms;
    return FD_OK;
}

}  // namespace fdh

using namespace fdh;

extern "C" {

int fd_autotune(const fd_grid* grid, int32_t nshot, const fd_opts* opts, int32_t steps,
                fd_opts* best, double* best_ms, void* stream)
{
    g_err.clear();
    return autotune(grid, nshot, opts, steps, best, best_ms, (hipStream_t)stream);
}

}  // extern "C"
