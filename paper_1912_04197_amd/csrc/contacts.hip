// Aggregate identification (subsection "Post-processing: aggregate
// identification"): bodies are the vertices of a graph whose edges are the
// contacts, and aggregates are its connected components with more than one
// body. The paper fills a contact container from its contact model and
// traverses the graph depth first; here the contacts are sphere overlaps
// found on the GPU with the Morton-sorted bodies of the tree build, and the
// components come from a lock-free union-find over those edges.
//
//   1. the cell level: the deepest tree level whose cell side is at least the
//      largest contact distance 2 r_max + skin, so every contact joins two
//      bodies in the same or adjacent cells of that level;
//   2. one thread per sorted body scans the bodies of the 27 cells around its
//      own (each cell a contiguous key range: a binary search for its start,
//      galloping from there for its end) and, for every body later in the
//      sorted order within r_s + r_t + skin, counts the contact and unites
//      the two bodies' sets; the radii are first gathered into sorted order;
//   3. union-find on caller indices: a set is named by its smallest index,
//      the larger of two roots is linked under the smaller with a
//      compare-and-swap, finds halve paths; parent[i] <= i always, so every
//      find ends, and a failed link is always another thread's success;
//   4. every body takes its root as label; roots of sets larger than one
//      body are counted.
#include "bhx_impl.h"

namespace bhx {
namespace {

__device__ inline int32_t load_fresh(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int32_t uf_find(int32_t *parent, int32_t x)
{
    for (;;) {
        const int32_t p = load_fresh(parent + x);
        if (p == x) return x;
        const int32_t gp = load_fresh(parent + p);
        if (gp != p) atomicCAS(parent + x, p, gp);  // path halving
        x = gp;
    }
}

__device__ inline void uf_union(int32_t *parent, int32_t a, int32_t b)
{
    for (;;) {
        a = uf_find(parent, a);
        b = uf_find(parent, b);
        if (a == b) return;
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(parent + a, a, b) == a) return;  // larger root under the smaller
    }
}

// counters: [0] contacts, [1] aggregates, [2] cell level, [3] bits of the
// largest radius (a non-negative double, so its bits order like the value)
__global__ __launch_bounds__(64) void k_contact_init(unsigned long long *__restrict__ counters)
{
    if (threadIdx.x < 4) counters[threadIdx.x] = 0ull;
}

__global__ __launch_bounds__(256) void k_radius_max(const double *__restrict__ radius, int64_t n,
                                                    unsigned long long *__restrict__ counters)
{
    __shared__ double red[4];
    double r = 0.0;  // fmax ignores NaN; negative radii never exceed 0
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        r = fmax(r, radius[i]);
    for (int o = 32; o > 0; o >>= 1) r = fmax(r, __shfl_xor(r, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        atomicMax(counters + 3, (unsigned long long)__double_as_longlong(r));
    }
}

__global__ __launch_bounds__(64) void k_contact_level(double skin, const SceneBox *__restrict__ box,
                                                      unsigned long long *__restrict__ counters)
{
    if (threadIdx.x != 0) return;
    const double r = __longlong_as_double((long long)counters[3]);
    const double reach = 2.0 * r + skin;
    int level = 0;
    while (level < kMaxLevel && ldexp(box[0].L, -(level + 1)) >= reach) level++;
    counters[2] = (unsigned long long)level;
}

__global__ __launch_bounds__(256) void k_uf_init(int32_t *__restrict__ label, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) label[i] = (int32_t)i;
}

// First sorted position whose key is >= k.
__device__ inline int64_t lower_bound(const uint64_t *__restrict__ keys, int64_t n, uint64_t k)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < k)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// First position >= from whose key is >= k, by doubling steps from `from`
// and a binary search in the last step (cheap when the answer is near).
__device__ inline int64_t gallop_lower_bound(const uint64_t *__restrict__ keys, int64_t from,
                                             int64_t n, uint64_t k)
{
    if (from >= n || keys[from] >= k) return from;
    int64_t lo = from, step = 1;  // keys[lo] < k
    while (lo + step < n && keys[lo + step] < k) {
        lo += step;
        step <<= 1;
    }
    int64_t hi = lo + step < n ? lo + step : n;  // keys[hi] >= k, or hi == n
    lo += 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < k)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Radii in sorted order (rs[s] = radius[idx[s]]), so the contact test reads
// them next to the bodies.
__global__ __launch_bounds__(256) void k_radius_sorted(const double *__restrict__ radius,
                                                       const uint32_t *__restrict__ idx, int64_t n,
                                                       double *__restrict__ rs)
{
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s < n) rs[s] = radius[idx[s]];
}

__global__ __launch_bounds__(256) void k_contacts(const Body *__restrict__ body,
                                                  const uint64_t *__restrict__ keys,
                                                  const uint32_t *__restrict__ idx,
                                                  const double *__restrict__ rsort, int64_t n,
                                                  double skin, int32_t *__restrict__ parent,
                                                  unsigned long long *__restrict__ counters)
{
#pragma clang fp contract(off)
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    unsigned long long found = 0;
    if (s < n) {
        const int level = (int)counters[2];
        const int drop = kMaxLevel - level;  // bits below the level's cell coordinate
        const uint64_t key = keys[s];
        const int32_t c[3] = {(int32_t)(compact3(key >> 2) >> drop),
                              (int32_t)(compact3(key >> 1) >> drop),
                              (int32_t)(compact3(key) >> drop)};
        const int32_t nside = 1 << level;
        const Body me = body[s];
        const double rs = rsort[s];
        int32_t is = -1;  // caller index, loaded at the first contact
        for (int dx = -1; dx <= 1; dx++) {
            const int32_t x = c[0] + dx;
            if (x < 0 || x >= nside) continue;
            for (int dy = -1; dy <= 1; dy++) {
                const int32_t y = c[1] + dy;
                if (y < 0 || y >= nside) continue;
                for (int dz = -1; dz <= 1; dz++) {
                    const int32_t z = c[2] + dz;
                    if (z < 0 || z >= nside) continue;
                    const uint64_t nb = (spread3((uint64_t)x) << 2) |
                                        (spread3((uint64_t)y) << 1) | spread3((uint64_t)z);
                    const int64_t lo = lower_bound(keys, n, nb << (3 * drop));
                    const int64_t hi = gallop_lower_bound(keys, lo, n, (nb + 1) << (3 * drop));
                    for (int64_t t = lo > s + 1 ? lo : s + 1; t < hi; t++) {
                        const Body o = body[t];
                        const double ex = o.x - me.x, ey = o.y - me.y, ez = o.z - me.z;
                        const double d2 = ex * ex + ey * ey + ez * ez;
                        const double R = rs + rsort[t] + skin;
                        if (d2 <= R * R) {
                            found++;
                            if (is < 0) is = (int32_t)idx[s];
                            uf_union(parent, is, (int32_t)idx[t]);
                        }
                    }
                }
            }
        }
    }
    // one atomic per wave on the contact counter
    for (int o = 32; o > 0; o >>= 1) found += __shfl_xor(found, o);
    if ((threadIdx.x & 63) == 0 && found) atomicAdd(counters, found);
}

__global__ __launch_bounds__(256) void k_size_clear(int32_t *__restrict__ size, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) size[i] = 0;
}

__global__ __launch_bounds__(256) void k_uf_flatten(int32_t *__restrict__ label, int64_t n,
                                                    int32_t *__restrict__ size)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int32_t r = uf_find(label, (int32_t)i);
    atomicAdd(size + r, 1);
}

__global__ __launch_bounds__(256) void k_uf_finish(int32_t *__restrict__ label, int64_t n,
                                                   const int32_t *__restrict__ size,
                                                   unsigned long long *__restrict__ counters)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool agg = false;
    if (i < n) {
        label[i] = uf_find(label, (int32_t)i);
        agg = size[i] > 1;
    }
    // one atomic per wave on the aggregate counter
    const uint64_t b = __ballot(agg);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(counters + 1, (unsigned long long)__popcll(b));
}

inline unsigned grid(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_contacts(const Workspace &w, hipStream_t s, const double *radius, int64_t n,
                           double skin, int32_t *label, int32_t *size,
                           unsigned long long *counters)
{
    if (n <= 0) return hipSuccess;
    k_contact_init<<<1, 64, 0, s>>>(counters);
    const unsigned rb = grid(n) < 1024u ? grid(n) : 1024u;
    k_radius_max<<<rb, 256, 0, s>>>(radius, n, counters);
    k_contact_level<<<1, 64, 0, s>>>(skin, w.box, counters);
    k_uf_init<<<grid(n), 256, 0, s>>>(label, n);
    // the sort's second key buffer is free after the build: sorted radii
    double *rsort = reinterpret_cast<double *>(w.keys[1]);
    k_radius_sorted<<<grid(n), 256, 0, s>>>(radius, w.idx[0], n, rsort);
    k_contacts<<<grid(n), 256, 0, s>>>(w.body, w.keys[0], w.idx[0], rsort, n, skin, label,
                                       counters);
    k_size_clear<<<grid(n), 256, 0, s>>>(size, n);
    k_uf_flatten<<<grid(n), 256, 0, s>>>(label, n, size);
    k_uf_finish<<<grid(n), 256, 0, s>>>(label, n, size, counters);
    return hipGetLastError();
}

}  // namespace bhx
