// Autotuner of the list kernels' launch shape (hough_hier_autotune).
//
// A workload class is the device (architecture, compute units, HIP runtime
// version) and the shape of a call (input kind, number of inputs, total
// pixels or points as a power of two, deepest level, variant, compare width,
// membership).  For a class not in the cache, each candidate shape runs the
// caller's sample call once to warm up and then twice timed (wall clock
// around the call, which waits for its results); the fastest is kept.  The
// cache is a small JSON object of class -> shape and time, rewritten whole
// (through a temporary file and a rename) after each new choice.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include <sys/stat.h>
#include <unistd.h>

#include "hh_engine.hpp"

namespace hh {

namespace {

struct Choice {
    int32_t task_steps = 8, queue_batch = 0, wg_per_cu = 0;
    double ms = 0.0;
};

std::string cache_path()
{
    if (const char* p = std::getenv("HH_TUNE_CACHE")) return p;
    const char* home = std::getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/hough_hier_tune.json";
}

// The cache file: {"<class>": {"task_steps": a, "queue_batch": b, "wg_per_cu": c, "ms": d}, ...}
// written by save() below; anything else in the file is ignored.
std::map<std::string, Choice> load(const std::string& path)
{
    std::map<std::string, Choice> m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t at = 0;
    for (;;) {
        const size_t k0 = s.find("\n  \"", at);
        if (k0 == std::string::npos) break;
        const size_t k1 = s.find('"', k0 + 4);
        const size_t b0 = s.find('{', k1), b1 = s.find('}', k1);
        if (k1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos) break;
        const std::string key = s.substr(k0 + 4, k1 - (k0 + 4));
        const std::string body = s.substr(b0, b1 - b0);
        auto num = [&](const char* name, double dflt) {
            const size_t p = body.find(std::string("\"") + name + "\":");
            return p == std::string::npos ? dflt : std::atof(body.c_str() + p + std::string(name).size() + 3);
        };
        Choice c;
        c.task_steps = (int32_t)num("task_steps", 4);
        c.queue_batch = (int32_t)num("queue_batch", 0);
        c.wg_per_cu = (int32_t)num("wg_per_cu", 0);
        c.ms = num("ms", 0.0);
        if (c.task_steps >= 1 && c.task_steps <= kMaxTaskSteps && c.queue_batch >= 0 && c.wg_per_cu >= 0)
            m[key] = c;
        at = b1;
    }
    return m;
}

void save(const std::string& path, const std::map<std::string, Choice>& m)
{
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) (void)mkdir(path.substr(0, slash).c_str(), 0755);
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    {
        std::ofstream f(tmp);
        if (!f) return;   // the cache is an optimisation: no file, no cache
        f << "{";
        bool first = true;
        for (const auto& kv : m) {
            f << (first ? "" : ",") << "\n  \"" << kv.first << "\": {\"task_steps\": " << kv.second.task_steps
              << ", \"queue_batch\": " << kv.second.queue_batch << ", \"wg_per_cu\": " << kv.second.wg_per_cu
              << ", \"ms\": " << kv.second.ms << "}";
            first = false;
        }
        f << "\n}\n";
    }
    (void)std::rename(tmp.c_str(), path.c_str());
}

int ceil_log2_u(int64_t n)
{
    int d = 0;
    while (((int64_t)1 << d) < n) ++d;
    return d;
}

std::string class_key(hh_ctx* ctx, const hh_input* in, int32_t n)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess) {
        (void)hipGetLastError();
        throw Error{HH_EDEVICE, "hipGetDeviceProperties failed"};
    }
    int rt = 0;
    (void)hipRuntimeGetVersion(&rt);
    int64_t size = 0;
    int32_t side = 1, depth = 0;
    for (int32_t k = 0; k < n; ++k) {
        size += in[k].kind == 0 ? in[k].n_points : (int64_t)in[k].width * in[k].height;
        side = std::max(side, std::max(in[k].width, in[k].height));
        const int32_t d = in[k].max_depth == INT32_MIN ? ctx->cfg.max_depth : in[k].max_depth;
        depth = std::max(depth, d == 0 ? ceil_log2_u(side) : std::max(d, 0));
    }
    std::ostringstream k;
    k << std::string(prop.gcnArchName).substr(0, 6) << "/cu" << prop.multiProcessorCount << "/hip" << rt << "/kind"
      << in[0].kind << "/n" << ceil_log2_u(n) << "/size" << ceil_log2_u(std::max<int64_t>(size, 1)) << "/d" << depth
      << "/v" << ctx->cfg.variant << "/w" << ((ctx->cfg.flags & HH_FLAG_WIDE_COMPARE) ? 64 : 32) << "/m"
      << ctx->cfg.membership << "/p" << ctx->cfg.passes;
    return k.str();
}

double time_call(hh_ctx* ctx, const hh_input* in, int32_t n)
{
    std::vector<hh_result*> out((size_t)n, nullptr);
    auto once = [&] {
        engine_detect_batch(ctx, in, n, out.data());
        for (hh_result* r : out) {
            {
                std::lock_guard<std::mutex> g(ctx->results_mu);
                ctx->live_results.erase(r);
                if (r->in_arena) --ctx->arena_results;
            }
            delete r;
        }
    };
    once();   // warm: arena sizes, groups
    double best = 1e30;
    for (int rep = 0; rep < 2; ++rep) {
        const auto t0 = std::chrono::steady_clock::now();
        once();
        best = std::min(best, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    }
    return best;
}

}  // namespace

hh_status engine_autotune(hh_ctx* ctx, const hh_input* in, int32_t n, hh_launch* chosen, int32_t* from_cache)
{
    const std::string key = class_key(ctx, in, n);
    const std::string path = cache_path();
    std::map<std::string, Choice> cache = load(path);
    Choice best;
    auto it = cache.find(key);
    *from_cache = it != cache.end() ? 1 : 0;
    if (it != cache.end()) {
        best = it->second;
    } else {
        static const int32_t kSteps[] = {1, 2, 4, 8, 16};
        static const int32_t kWg[] = {0, 4};
        best.ms = 1e30;
        for (int32_t steps : kSteps)
            for (int32_t wg : kWg) {
                ctx->task_steps = steps;
                ctx->queue_batch = 0;
                ctx->wg_per_cu = wg;
                const double ms = time_call(ctx, in, n);
                if (ms < best.ms) best = Choice{steps, 0, wg, ms};
            }
        cache = load(path);   // another process may have written meanwhile
        cache[key] = best;
        save(path, cache);
    }
    ctx->task_steps = best.task_steps;
    ctx->queue_batch = best.queue_batch;
    ctx->wg_per_cu = best.wg_per_cu;
    chosen->task_steps = best.task_steps;
    chosen->queue_batch = best.queue_batch;
    chosen->wg_per_cu = best.wg_per_cu;
    chosen->reserved = 0;
    return HH_OK;
}

}  // namespace hh
