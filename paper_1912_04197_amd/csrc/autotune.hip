// Autotuner for batched stepping: picks the bucket size (leaf) and the walk
// group size that make bh_batched_step fastest on a given set of scenes.
//
// Every candidate gets its own context (sized for the layout) and scratch
// copies of the caller's state, so the caller's arrays are never modified.
// A candidate is warmed up by one graph-captured step and then timed over
// `steps` replays with HIP events on its stream. Results can be cached in a
// file of JSON lines named by the BHX_AUTOTUNE_CACHE environment variable,
// keyed by the layout and the physical parameters.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "bhx_impl.h"

namespace {

std::string cache_key(const bh_config *base, int32_t n_scenes, const int64_t *offsets,
                      double softening, bool per_body_eps, double theta, double dt)
{
    // layout digest: FNV-1a over the offsets
    uint64_t h = 1469598103934665603ull;
    for (int32_t k = 0; k <= n_scenes; k++) {
        uint64_t v = (uint64_t)offsets[k];
        for (int b = 0; b < 8; b++) {
            h ^= (v >> (8 * b)) & 0xff;
            h *= 1099511628211ull;
        }
    }
    char buf[256];
    // flags that change the timed kernels (quadrupole nodes) are part of the key
    const unsigned kflags = base->flags & (uint32_t)BH_FLAG_QUAD;
    std::snprintf(buf, sizeof buf, "scenes=%d;n=%lld;layout=%016llx;prec=%d;flags=%u;G=%.17g;"
                                   "soft=%.17g;eps=%d;theta=%.17g;dt=%.17g",
                  n_scenes, (long long)offsets[n_scenes], (unsigned long long)h, base->precision,
                  kflags, base->G, softening, per_body_eps ? 1 : 0, theta, dt);
    return buf;
}

bool cache_lookup(const std::string &key, bh_tune_result *out)
{
    const char *path = std::getenv("BHX_AUTOTUNE_CACHE");
    if (!path || !*path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        const std::string s(line);
        const std::string tag = "\"key\": \"" + key + "\"";
        if (s.find(tag) == std::string::npos) continue;
        int leaf = 0, group = 0;
        double ms = 0.0;
        const size_t a = s.find("\"leaf\": "), b = s.find("\"group\": "), c = s.find("\"ms\": ");
        if (a == std::string::npos || b == std::string::npos || c == std::string::npos) continue;
        if (std::sscanf(s.c_str() + a + 8, "%d", &leaf) == 1 &&
            std::sscanf(s.c_str() + b + 9, "%d", &group) == 1 &&
            std::sscanf(s.c_str() + c + 6, "%lf", &ms) == 1) {
            out->leaf_size = leaf;
            out->walk_group = group;
            out->ms_per_step = ms;
            found = true;  // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const std::string &key, const bh_tune_result &r)
{
    const char *path = std::getenv("BHX_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "{\"key\": \"%s\", \"leaf\": %d, \"group\": %d, \"ms\": %.17g}\n", key.c_str(),
                 r.leaf_size, r.walk_group, r.ms_per_step);
    std::fclose(f);
}

}  // namespace

extern "C" bh_status bh_autotune(const bh_config *base, void *hip_stream, int32_t n_scenes,
                                 const int64_t *offsets, const double *pos, const double *vel,
                                 const double *mass, double softening, const double *eps,
                                 double theta, double dt, int32_t steps, bh_tune_result *out)
{
    if (!base || !offsets || !out || !pos || !vel || !mass) return BH_E_INVALID;
    if (n_scenes < 1 || steps < 1 || !(theta >= 0.0) || !std::isfinite(theta) ||
        !std::isfinite(dt))
        return BH_E_INVALID;
    const int64_t n = offsets[n_scenes];
    if (n < 1) return BH_E_INVALID;
    const std::string key = cache_key(base, n_scenes, offsets, softening, eps != nullptr, theta, dt);
    if (cache_lookup(key, out)) return BH_OK;

    hipStream_t caller = (hipStream_t)hip_stream;
    if (hipStreamSynchronize(caller) != hipSuccess) return BH_E_HIP;
    double *p = nullptr, *v = nullptr, *a = nullptr;
    const size_t bytes = (size_t)n * 3 * sizeof(double);
    if (hipMalloc((void **)&p, bytes) != hipSuccess || hipMalloc((void **)&v, bytes) != hipSuccess ||
        hipMalloc((void **)&a, bytes) != hipSuccess) {
        (void)hipFree(p);
        (void)hipFree(v);
        (void)hipFree(a);
        return BH_E_OOM;
    }
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bh_status status = BH_OK;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        status = BH_E_HIP;

    const int leaves[] = {4, 8, 16, 32};
    const int groups[] = {16, 32, 64};
    bh_tune_result best{0, 0, INFINITY};
    for (int leaf : leaves) {
        for (int group : groups) {
            if (status) break;
            bh_config cfg = *base;
            cfg.n_max = n;
            cfg.leaf_size = leaf;
            cfg.walk_group = group;
            cfg.max_scenes = n_scenes;
            cfg.flags = (base->flags & ~(uint32_t)(BH_FLAG_COUNTS | BH_FLAG_TIMING | BH_FLAG_ADJOINT)) |
                        BH_FLAG_GRAPH;
            bh_ctx *c = nullptr;
            bh_status r = bh_create(&cfg, s, &c);
            if (r == BH_E_OOM) continue;  // a candidate that does not fit is skipped
            if (r) {
                status = r;
                break;
            }
            float ms = 0.f;
            if (hipMemcpyAsync(p, pos, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
                hipMemcpyAsync(v, vel, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
                r = BH_E_HIP;
            if (!r) r = bh_batched_accel(c, n_scenes, offsets, p, mass, softening, eps, theta, a, nullptr);
            if (!r) r = bh_batched_step(c, n_scenes, offsets, p, v, mass, softening, eps, theta, dt, 1, a);
            if (!r && hipEventRecord(e0, s) != hipSuccess) r = BH_E_HIP;
            if (!r) r = bh_batched_step(c, n_scenes, offsets, p, v, mass, softening, eps, theta, dt, steps, a);
            if (!r && hipEventRecord(e1, s) != hipSuccess) r = BH_E_HIP;
            if (!r) r = bh_sync(c);
            if (!r && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) r = BH_E_HIP;
            bh_destroy(c);
            if (r) {
                status = r;
                break;
            }
            const double per = (double)ms / steps;
            if (per < best.ms_per_step) best = bh_tune_result{leaf, group, per};
        }
    }
    if (s) (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(p);
    (void)hipFree(v);
    (void)hipFree(a);
    if (status) return status;
    if (!(best.leaf_size > 0)) return BH_E_OOM;
    *out = best;
    cache_store(key, best);
    return BH_OK;
}
