// Autotuner for the launch shapes of the hot kernels.
//
// Pair kernel: test points per lane (1 or 2) and the number of trial splits
// (workgroups per test block).  GEMM: the number of K slices.  Every candidate
// runs on the problem's own data, timed with HIP events on its stream
// (median of a few launches); the fastest wins.  Choices are cached in
// memory per process and in a small text file (path from BEM_TUNE_CACHE,
// default ~/.cache/bem_mi355x_tune.txt; one "key value" line per choice, the
// last line of a key wins) keyed by GPU architecture, kernel, size bucket and
// precision, so a later problem of the same bucket skips the search.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "bem_internal.h"

namespace bem {

namespace {

std::mutex g_mu;
std::map<std::string, int> g_cache;
std::string g_loaded;   // path the in-memory cache was read from
// bumped whenever a tuned kernel changes, so that older choices are not reused
constexpr const char *TUNE_VERSION = "v2";

std::string cache_path()
{
    if (const char *e = std::getenv("BEM_TUNE_CACHE")) return e;
    const char *home = std::getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/bem_mi355x_tune.txt";
}

// (Re)read the cache file when the configured path changes.
void load_cache()
{
    const std::string path = cache_path();
    if (path == g_loaded) return;
    g_loaded = path;
    g_cache.clear();
    std::ifstream f(path);
    std::string k;
    int v;
    while (f >> k >> v) g_cache[k] = v;
}

void store(const std::string &key, int value)
{
    g_cache[key] = value;
    std::ofstream f(cache_path(), std::ios::app);
    if (f) f << key << " " << value << "\n";
}

std::string arch_name(int device)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    return a.substr(0, a.find(':'));
}

int bucket(int64_t x)
{
    int b = 0;
    while ((int64_t(1) << (b + 1)) <= x) ++b;
    return b;
}

template <typename F>
float time_ms(bem_problem &p, F &&launch, int reps)
{
    hipEvent_t a, b;
    BEM_HIP(hipEventCreate(&a));
    BEM_HIP(hipEventCreate(&b));
    launch();   // warm
    std::vector<float> ts;
    for (int r = 0; r < reps; ++r) {
        BEM_HIP(hipEventRecord(a, p.stream));
        launch();
        BEM_HIP(hipEventRecord(b, p.stream));
        BEM_HIP(hipEventSynchronize(b));
        float ms = 0;
        BEM_HIP(hipEventElapsedTime(&ms, a, b));
        ts.push_back(ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    std::sort(ts.begin(), ts.end());
    return ts[ts.size() / 2];
}

}  // namespace

// Choose (test points per lane, trial splits) of the pair kernel; rebuilds the
// work list.  Returns the chosen code 100 * tpl + n_split.
int tune_pairs(bem_problem &p, void (*rebuild)(bem_problem &), int max_split)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache();
    std::ostringstream key;
    key << "pairs" << TUNE_VERSION << ":" << arch_name(p.device) << ":M" << bucket(p.M) << ":P" << p.n_pass;
    auto it = g_cache.find(key.str());
    const auto valid = [&](int code) {
        const int tpl = code / 100, ns = code % 100;
        return (tpl == 1 || tpl == 2) && ns >= 1 && ns <= max_split;
    };
    if (it != g_cache.end() && valid(it->second)) {
        p.tpl = it->second / 100;
        p.n_split = it->second % 100;
        rebuild(p);
        return it->second;
    }
    // trial data for the timing: the gather of a constant vector
    double2 *x = nullptr;
    BEM_HIP(hipMallocAsync(reinterpret_cast<void **>(&x), size_t(p.N) * sizeof(double2), p.stream));
    BEM_HIP(hipMemsetAsync(x, 0, size_t(p.N) * sizeof(double2), p.stream));
    launch_gather(p, x);
    const int64_t blocks = (p.M + 255) / 256;
    std::vector<std::pair<float, int>> timed;   // (ms, code)
    const auto run = [&](int code, int reps) {
        p.tpl = code / 100;
        p.n_split = code % 100;
        rebuild(p);
        // the partial sums of every split are read back by the reduction: time both
        return time_ms(p, [&]() { launch_pairs(p); launch_reduce(p); }, reps);
    };
    bool warmed = false;
    for (int tpl : {1, 2}) {
        for (int ns : {1, 2, 4, 8, 16, 32, 64}) {
            const int64_t wgs = int64_t(p.n_pass) * ((blocks + tpl - 1) / tpl) * ns;
            if (wgs < 256 || wgs > (int64_t(1) << 22)) continue;   // too few to fill 256 CUs / absurdly many
            if (int64_t(ns) * 256 > p.M || ns > max_split) continue;
            const int code = 100 * tpl + ns;
            if (!warmed) {
                // bring the clocks to their loaded state before the first timing
                for (int w = 0; w < 4; ++w) (void)run(code, 1);
                warmed = true;
            }
            timed.emplace_back(run(code, p.M > 200000 ? 1 : 3), code);
        }
    }
    // second pass: the three fastest candidates again, interleaved, so that a
    // drift of the clock during the sweep does not decide between near-equal shapes
    std::sort(timed.begin(), timed.end());
    int best = 0;
    if (!timed.empty()) {
        const size_t nb = std::min<size_t>(3, timed.size());
        std::vector<std::vector<float>> again(nb);
        for (int round = 0; round < 3; ++round)
            for (size_t c = 0; c < nb; ++c) again[c].push_back(run(timed[c].second, 1));
        float best_ms = 1e30f;
        for (size_t c = 0; c < nb; ++c) {
            std::sort(again[c].begin(), again[c].end());
            if (again[c][1] < best_ms) {
                best_ms = again[c][1];
                best = timed[c].second;
            }
        }
    }
    (void)hipFreeAsync(x, p.stream);
    if (best == 0) best = 100 + std::max(1, std::min(max_split, int(std::min<int64_t>(64, (2048 + blocks - 1) / std::max<int64_t>(1, blocks)))));
    p.tpl = best / 100;
    p.n_split = best % 100;
    rebuild(p);
    store(key.str(), best);
    return best;
}

std::string gemm_key(const bem_problem &p, int R, bool bf16)
{
    std::ostringstream key;
    key << "gemm" << TUNE_VERSION << ":" << arch_name(p.device) << ":N" << bucket(p.N) << ":R" << bucket(R) << ":" << (bf16 ? "bf16x3d" : "f32c");
    return key.str();
}

// Codes of the GEMM choice: 100 * tile shape + K slices.
static bool valid_gemm_code(int code, bool bf16)
{
    const int shape = code / 100, ns = code % 100;
    return ns >= 1 && ns <= 64 && (shape == 0 || (bf16 && shape == 1));
}

int cached_gemm_slices(bem_problem &p, int R, bool bf16)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache();
    auto it = g_cache.find(gemm_key(p, R, bf16));
    return it != g_cache.end() && valid_gemm_code(it->second, bf16) ? it->second : 0;
}

// Tile shape and number of K slices of the GEMM for R right-hand sides, tuned
// once per bucket; returns the code 100 * shape + slices.
int tune_gemm_slices(bem_problem &p, int R, bool bf16, void *xbuf, float *cbuf, double2 *Y)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache();
    const std::string key = gemm_key(p, R, bf16);
    auto it = g_cache.find(key);
    if (it != g_cache.end() && valid_gemm_code(it->second, bf16) &&
        gemm_plan(p, R, bf16, it->second % 100, it->second / 100).bytes_c <= p.gc_bytes)
        return it->second;
    int best = gemm_plan(p, R, bf16, 0).n_s;
    float best_ms = 1e30f;
    for (int shape = 0; shape < (bf16 ? 2 : 1); ++shape) {
        for (int s : {1, 2, 4, 8, 16, 32, 64}) {
            const GemmPlan g = gemm_plan(p, R, bf16, s, shape);
            if (g.bytes_c > p.gc_bytes || g.bytes_x > p.gx_bytes) continue;
            // the slice count trades GEMM occupancy against partials to sum: time both
            const float ms = time_ms(p, [&]() {
                launch_gemm_kernel(p, g, xbuf, cbuf);
                launch_unpack(p, g, cbuf, Y);
            }, 2);
            if (ms < best_ms) {
                best_ms = ms;
                best = 100 * shape + g.n_s;
            }
        }
    }
    store(key, best);
    return best;
}

}  // namespace bem
