// Octree construction on the device, rebuilt on every force evaluation
// (subsection "Hierarchical treecode algorithm"; the five GPU stages of
// subsection "CUDA implementation of GPU-parallel Barnes-Hut" are prior art,
// this is a Morton-key design for CDNA4):
//   1. bounding box of each scene's bodies -> its root cube (and input
//      validation); a call may hold many independent scenes, stored as
//      contiguous body ranges, each with its own root,
//   2. 63-bit Morton keys on a 2^21 grid,
//   3. stable LSD radix sort of (key, index), 8-bit digits, LDS ranking, then
//      (several scenes) two stable passes on the scene index,
//   4. gather of positions, masses and softening into Morton order,
//   5. top-down octree, one launch per level: each split cell finds its
//      octant ranges by binary search in the sorted keys,
//   6. bottom-up moments, one launch per level: mass and centre of mass from
//      the children by eq. (COMinternal), leaves from their bodies.
// Every launch reads its sizes from the device tree header, so the sequence
// needs no host round trip and can be captured in a graph.
#include <cmath>

#include "bhx_impl.h"

namespace bhx {
namespace {

constexpr double kInf = __builtin_huge_val();

__device__ inline uint64_t lanemask_lt(int lane) { return (1ull << lane) - 1ull; }

template <typename T>
__device__ inline T wave_min(T v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
template <typename T>
__device__ inline T wave_max(T v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Inclusive scan over a 256-thread block (4 waves).
__device__ inline uint32_t block_incl_scan_256(uint32_t v, uint32_t *lds4, uint32_t *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_incl_scan(v);
    if (lane == 63) lds4[wave] = v;
    __syncthreads();
    uint32_t add = 0, tot = 0;
    for (int w = 0; w < 4; w++) {
        uint32_t x = lds4[w];
        if (w < wave) add += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return v + add;
}

// ---------------------------------------------------------------- 1. box

// Order-preserving map of doubles to unsigned integers, so integer atomics
// give the exact minimum and maximum whatever the order of the updates.
__device__ inline unsigned long long order_enc(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ inline double order_dec(unsigned long long e)
{
    const unsigned long long b = (e >> 63) ? (e & 0x7fffffffffffffffull) : ~e;
    return __longlong_as_double((long long)b);
}

__global__ __launch_bounds__(256) void k_box_init(SceneBox *__restrict__ box, int n_scenes)
{
    const int sc = blockIdx.x * 256 + threadIdx.x;
    if (sc >= n_scenes) return;
    for (int a = 0; a < 3; a++) {
        box[sc].lo_enc[a] = ~0ull;
        box[sc].hi_enc[a] = 0ull;
    }
}

// One work item: a chunk of at most kBoxChunk bodies of one scene (for one
// scene, chunk c is bodies c*kBoxChunk onwards). Reduces its box in the block
// and merges it into the scene's with integer atomics; flags bad input.
constexpr int kBoxThreads = 1024;  // one block per chunk: 4 bodies per thread
__global__ __launch_bounds__(kBoxThreads) void k_box_chunk(const double *__restrict__ pos,
                                                   const double *__restrict__ mass,
                                                   const double *__restrict__ eps, int64_t n,
                                                   const int32_t *__restrict__ chunks,
                                                   SceneBox *__restrict__ box,
                                                   TreeHeader *__restrict__ hdr)
{
    int sc = 0;
    int64_t first = (int64_t)blockIdx.x * kBoxChunk, end = first + kBoxChunk;
    if (chunks) {
        sc = chunks[3 * blockIdx.x];
        first = chunks[3 * blockIdx.x + 1];
        end = chunks[3 * blockIdx.x + 2];
    }
    if (end > n) end = n;
    double lo[3] = {kInf, kInf, kInf}, hi[3] = {-kInf, -kInf, -kInf};
    bool bad = false;
    for (int64_t i = first + threadIdx.x; i < end; i += kBoxThreads) {
        double x[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
        double m = mass[i];
        bad |= !(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]));
        bad |= !(isfinite(m) && m >= 0.0);
        if (eps) {
            double e = eps[i];
            bad |= !(isfinite(e) && e >= 0.0);
        }
        for (int a = 0; a < 3; a++) {
            lo[a] = fmin(lo[a], x[a]);
            hi[a] = fmax(hi[a], x[a]);
        }
    }
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&hdr->status, ST_NONFINITE);
    __shared__ double red[kBoxThreads / 64][6];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int a = 0; a < 3; a++) {
        double l = wave_min(lo[a]), h = wave_max(hi[a]);
        if (lane == 0) {
            red[wave][a] = l;
            red[wave][3 + a] = h;
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int a = threadIdx.x;
        double v = red[0][a];
        for (int w = 1; w < kBoxThreads / 64; w++)
            v = a < 3 ? fmin(v, red[w][a]) : fmax(v, red[w][a]);
        if (a < 3)
            atomicMin(&box[sc].lo_enc[a], order_enc(v));
        else
            atomicMax(&box[sc].hi_enc[a - 3], order_enc(v));
    }
}

// The same work items for one step of a multi-step call, on the sorted state
// of the previous build: kick and drift each body (v = v + (dt/2) a, then
// x = x + dt v, each one fused multiply-add as the caller-order step rounds
// it), write the new state in the same order to the S buffers with its mass,
// softening and caller index, and reduce the box of the new positions.
__global__ __launch_bounds__(kBoxThreads) void k_state_kick_drift(
    const Body *__restrict__ body, const double *__restrict__ tvel,
    const double *__restrict__ tacc, const double *__restrict__ beps2,
    const uint32_t *__restrict__ cidx, int64_t n, double h, double dt,
    const int32_t *__restrict__ chunks, Body *__restrict__ sbody, double *__restrict__ svel,
    double *__restrict__ seps2, uint32_t *__restrict__ scidx, SceneBox *__restrict__ box,
    TreeHeader *__restrict__ hdr)
{
    int sc = 0;
    int64_t first = (int64_t)blockIdx.x * kBoxChunk, end = first + kBoxChunk;
    if (chunks) {
        sc = chunks[3 * blockIdx.x];
        first = chunks[3 * blockIdx.x + 1];
        end = chunks[3 * blockIdx.x + 2];
    }
    if (end > n) end = n;
    double lo[3] = {kInf, kInf, kInf}, hi[3] = {-kInf, -kInf, -kInf};
    bool bad = false;
    for (int64_t i = first + threadIdx.x; i < end; i += kBoxThreads) {
        const Body b = body[i];
        const double x0[3] = {b.x, b.y, b.z};
        double x[3], v[3];
        for (int a = 0; a < 3; a++) {
            v[a] = fma(h, tacc[3 * i + a], tvel[3 * i + a]);
            x[a] = fma(dt, v[a], x0[a]);
        }
        sbody[i] = Body{x[0], x[1], x[2], b.m};
        for (int a = 0; a < 3; a++) svel[3 * i + a] = v[a];
        if (seps2) seps2[i] = beps2[i];
        scidx[i] = cidx[i];
        bad |= !(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]));
        for (int a = 0; a < 3; a++) {
            lo[a] = fmin(lo[a], x[a]);
            hi[a] = fmax(hi[a], x[a]);
        }
    }
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&hdr->status, ST_NONFINITE);
    __shared__ double red[kBoxThreads / 64][6];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int a = 0; a < 3; a++) {
        double l = wave_min(lo[a]), hv = wave_max(hi[a]);
        if (lane == 0) {
            red[wave][a] = l;
            red[wave][3 + a] = hv;
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int a = threadIdx.x;
        double v = red[0][a];
        for (int w = 1; w < kBoxThreads / 64; w++)
            v = a < 3 ? fmin(v, red[w][a]) : fmax(v, red[w][a]);
        if (a < 3)
            atomicMin(&box[sc].lo_enc[a], order_enc(v));
        else
            atomicMax(&box[sc].hi_enc[a - 3], order_enc(v));
    }
}

// Root cube: side = largest extent (1 if all bodies coincide), centred on the
// bounding box; the quantisation scale and the squared cell side per level.
__device__ inline void root_cube(SceneBox &b, const double lo[3], const double hi[3])
{
#pragma clang fp contract(off)
    double L = 0.0;
    for (int a = 0; a < 3; a++) {
        double e = hi[a] - lo[a];
        if (e > L) L = e;
    }
    if (L == 0.0) L = 1.0;
    for (int a = 0; a < 3; a++) {
        b.lo[a] = lo[a];
        b.hi[a] = hi[a];
        b.x0[a] = (lo[a] + hi[a]) * 0.5 - L * 0.5;
    }
    b.L = L;
    b.S = 2097152.0 / L;
    for (int l = 0; l < kLevels; l++) {
        double sd = ldexp(L, -l);
        b.s2[l] = sd * sd;
    }
}

// Root cube of a scene into `out` from the reduced box encodings of `in`
// (the same SceneBox or a copy); a scene without bodies gets the cube at 0.
__device__ inline void scene_root_cube(SceneBox &out, const SceneBox &in, bool any)
{
    double lo[3], hi[3];
    for (int a = 0; a < 3; a++) {
        lo[a] = any ? order_dec(in.lo_enc[a]) : 0.0;
        hi[a] = any ? order_dec(in.hi_enc[a]) : 0.0;
    }
    root_cube(out, lo, hi);
}

// One thread per scene: root cube from the box, and the scene's root node
// (level 0, its bodies' whole range in sorted order). Thread 0 also resets
// the per-level node counts.
__global__ __launch_bounds__(256) void k_box_final(SceneBox *__restrict__ box, int n_scenes,
                                                   const int64_t *__restrict__ offsets, int64_t n,
                                                   TreeHeader *__restrict__ hdr,
                                                   NodeInfo *__restrict__ ninfo)
{
#pragma clang fp contract(off)
    const int sc = blockIdx.x * 256 + threadIdx.x;
    if (sc == 0) {
        for (int l = 0; l <= kLevels; l++) hdr->level_count[l] = 0;
        hdr->level_count[0] = n > 0 ? n_scenes : 0;
        hdr->cell_max = 0;
    }
    if (sc >= n_scenes) return;
    const int64_t first = offsets ? offsets[sc] : 0, end = offsets ? offsets[sc + 1] : n;
    SceneBox &b = box[sc];
    scene_root_cube(b, b, end > first);
    if (end > first)
        ninfo[sc] = NodeInfo{(int32_t)first, (int32_t)(end - first), -1, (int32_t)(sc << 16)};
}

// --------------------------------------------------------------- 2. keys

// Integer cell coordinate: clamp(floor((x - x0) * S), 0, 2^21 - 1), rounded
// exactly as written so every implementation of the cell definition agrees.
__device__ inline uint32_t quantise(double x, double x0, double S)
{
#pragma clang fp contract(off)
    double f = floor((x - x0) * S);
    if (!(f >= 0.0)) return 0u;
    if (f > (double)kQMax) return kQMax;
    return (uint32_t)f;
}

__device__ inline uint64_t morton_key(const double *x, const SceneBox &b)
{
    const uint32_t qx = quantise(x[0], b.x0[0], b.S);
    const uint32_t qy = quantise(x[1], b.x0[1], b.S);
    const uint32_t qz = quantise(x[2], b.x0[2], b.S);
    return (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
}

// pos: body i's coordinates at pos + stride * i (3: caller arrays, 4: Body)
__global__ __launch_bounds__(256) void k_keys(const double *__restrict__ pos, int stride, int64_t n,
                                              const SceneBox *__restrict__ box,
                                              const uint16_t *__restrict__ scene_of,
                                              uint64_t *__restrict__ keys,
                                              uint32_t *__restrict__ idx)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    keys[i] = morton_key(pos + stride * i, box[scene_of ? scene_of[i] : 0]);
    idx[i] = (uint32_t)i;
}

// --------------------------------------------------------------- 3. sort

// Scene index of caller index v: for at most kLdsScenes scenes a binary
// search of the scene offsets staged in LDS (soff), else scene_of[v].
constexpr int kLdsScenes = 256;
__device__ inline uint32_t scene_index(const int64_t *soff, int ns,
                                       const uint16_t *__restrict__ scene_of, uint32_t v)
{
    if (ns > kLdsScenes) return scene_of[v];
    int lo = 0, hi = ns;  // soff[lo] <= v < soff[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (soff[mid] <= (int64_t)v)
            lo = mid;
        else
            hi = mid;
    }
    return (uint32_t)lo;
}

// Sort digit of one element: 8 bits of its key, or for shift >= 64 8 bits of
// its scene index (shift - 64 = 0 or 8).
__device__ inline uint32_t sort_digit(uint64_t key, uint32_t val, int shift, const int64_t *soff,
                                      int ns, const uint16_t *__restrict__ scene_of)
{
    if (shift < 64) return (uint32_t)(key >> shift) & 255u;
    return (scene_index(soff, ns, scene_of, val) >> (shift - 64)) & 255u;
}

// Stages the scene offsets in LDS for the scene passes (before a barrier).
__device__ inline void stage_offsets(int64_t *soff, const int64_t *__restrict__ offsets, int ns,
                                     int shift)
{
    if (shift >= 64 && ns <= kLdsScenes)
        for (int i = threadIdx.x; i <= ns; i += blockDim.x) soff[i] = offsets[i];
}

// Per-tile digit histogram, written digit-major: counts[d * nblk + tile].
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const uint64_t *__restrict__ keys,
                                                            const uint32_t *__restrict__ vals,
                                                            const uint16_t *__restrict__ scene_of,
                                                            const int64_t *__restrict__ offsets,
                                                            int ns, int64_t n, int shift,
                                                            uint32_t *__restrict__ counts,
                                                            int nblk)
{
    __shared__ uint32_t h[256];
    __shared__ int64_t soff[kLdsScenes + 1];
    h[threadIdx.x] = 0;
    stage_offsets(soff, offsets, ns, shift);
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; r++) {
        int64_t i = base + r * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[sort_digit(keys[i], vals[i], shift, soff, ns, scene_of)], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of one digit's row of tile counts; one block per digit.
// k_box_final and k_keys for one scene, with the tile layout of k_sort_hist,
// and that kernel's digit counts of the first pass (bits shift..shift+7) of
// the same tile.
__global__ __launch_bounds__(kSortThreads) void k_keys_hist(const double *__restrict__ pos,
                                                            int stride, int64_t n,
                                                            SceneBox *__restrict__ box,
                                                            TreeHeader *__restrict__ hdr,
                                                            NodeInfo *__restrict__ ninfo,
                                                            uint64_t *__restrict__ keys,
                                                            uint32_t *__restrict__ idx, int shift,
                                                            uint32_t *__restrict__ counts,
                                                            int nblk)
{
#pragma clang fp contract(off)
    __shared__ uint32_t h[256];
    __shared__ SceneBox b;  // this block's copy of the root cube
    h[threadIdx.x] = 0;
    // k_box_final's work for the one scene (n > 0): every block computes the
    // root cube from the reduced box for itself, block 0 also stores it, the
    // level counts and the root node (no block reads those fields here)
    if (threadIdx.x == 0) {
        scene_root_cube(b, box[0], true);
        if (blockIdx.x == 0) {
            scene_root_cube(box[0], box[0], true);
            for (int l = 0; l <= kLevels; l++) hdr->level_count[l] = 0;
            hdr->level_count[0] = 1;
            hdr->cell_max = 0;
            ninfo[0] = NodeInfo{0, (int32_t)n, -1, 0};
        }
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; r++) {
        const int64_t i = base + r * kSortThreads + threadIdx.x;
        if (i < n) {
            const uint64_t key = morton_key(pos + stride * i, b);
            keys[i] = key;
            idx[i] = (uint32_t)i;
            atomicAdd(&h[(uint32_t)(key >> shift) & 255u], 1u);
        }
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_sort_scan(uint32_t *__restrict__ counts,
                                                   uint32_t *__restrict__ totals, int nblk)
{
    __shared__ uint32_t lds4[4];
    uint32_t *row = counts + (int64_t)blockIdx.x * nblk;
    uint32_t carry = 0;
    for (int b0 = 0; b0 < nblk; b0 += 256) {
        int b = b0 + threadIdx.x;
        uint32_t v = b < nblk ? row[b] : 0u, tot;
        uint32_t incl = block_incl_scan_256(v, lds4, &tot);
        if (b < nblk) row[b] = carry + incl - v;
        carry += tot;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Stable scatter of one tile. Wave w holds the tile's keys w*512 .. w*512+511
// (round r, lane l: key w*512 + r*64 + l, so tile order is (wave, round,
// lane) order). Each wave ranks its keys among equal digits with ballots and
// a per-wave digit count in LDS, without block barriers; one exclusive scan
// over the waves and one over the digits then place every key in a copy of
// the tile reordered by digit, so that consecutive threads write consecutive
// addresses of each digit's output run.
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    const uint16_t *__restrict__ scene_of, const int64_t *__restrict__ offsets, int ns,
    uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n, int shift,
    const uint32_t *__restrict__ counts, const uint32_t *__restrict__ totals, int nblk)
{
    static_assert(kSortThreads == 256 && kSortItems == 8, "four waves of eight rounds");
    constexpr int kWaveKeys = 64 * kSortItems;
    __shared__ uint32_t digit_base[256];
    __shared__ uint32_t whist[4][256];  // per-wave digit counts, then per-wave digit offsets
    __shared__ uint32_t lds4[4];
    __shared__ uint32_t lstart[256];
    __shared__ uint64_t skey[kSortTile];
    __shared__ uint32_t sval[kSortTile];
    __shared__ uint8_t sdig[kSortTile];  // digits of the reordered tile
    __shared__ int64_t soff[kLdsScenes + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    stage_offsets(soff, offsets, ns, shift);  // read after the barrier below

    uint32_t tot;
    const uint32_t t = totals[tid];
    const uint32_t incl = block_incl_scan_256(t, lds4, &tot);
    digit_base[tid] = incl - t + counts[(int64_t)tid * nblk + blockIdx.x];
    for (int w = 0; w < 4; w++) whist[w][tid] = 0;
    __syncthreads();

    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const int64_t wbase = base + wave * kWaveKeys;
    uint64_t k[kSortItems];
    uint32_t v[kSortItems], rank[kSortItems], dig[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const int64_t i = wbase + r * 64 + lane;
        k[r] = i < n ? kin[i] : 0ull;
        v[r] = i < n ? vin[i] : 0u;
    }
    uint32_t *const wh = whist[wave];
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const bool valid = wbase + r * 64 + lane < n;
        const uint32_t d = valid ? sort_digit(k[r], v[r], shift, soff, ns, scene_of) : 0u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const uint64_t lower = peers & lanemask_lt(lane);
        // keys of this digit ranked by earlier rounds of this wave, read by
        // every peer before the lowest one adds this round's peers
        const uint32_t before = valid ? wh[d] : 0u;
        if (valid && lower == 0) wh[d] = before + (uint32_t)__popcll(peers);
        rank[r] = before + (uint32_t)__popcll(lower);
        dig[r] = d;
    }
    __syncthreads();
    // digit tid: exclusive offsets of the waves, and its total in the tile
    {
        uint32_t run = 0;
        for (int w = 0; w < 4; w++) {
            const uint32_t c = whist[w][tid];
            whist[w][tid] = run;
            run += c;
        }
        uint32_t ctot;
        const uint32_t ci = block_incl_scan_256(run, lds4, &ctot);
        lstart[tid] = ci - run;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        if (wbase + r * 64 + lane < n) {
            const uint32_t lp = lstart[dig[r]] + wh[dig[r]] + rank[r];
            if (lp < (uint32_t)kSortTile) {
                skey[lp] = k[r];
                sval[lp] = v[r];
                sdig[lp] = (uint8_t)dig[r];
            }
        }
    }
    __syncthreads();
    const int cnt = (int)(n - base < kSortTile ? n - base : kSortTile);
    for (int lp = tid; lp < cnt; lp += kSortThreads) {
        const uint64_t key = skey[lp];
        const uint32_t val = sval[lp];
        const uint32_t d = sdig[lp];
        const int64_t o = (int64_t)digit_base[d] + lp - lstart[d];
        if (o >= 0 && o < n) {
            kout[o] = key;
            vout[o] = val;
        }
    }
}

// ------------------------------------------------------- 3b. bucket sort

// One scene: two stable passes on the top 16 key bits (bits 47..62) group the
// keys by bucket (equal top bits), in input order within each bucket; then
// one block per tile of sorted positions takes the buckets that start in its
// tile (through the end of the last one) and sorts them by the whole key,
// stably: in LDS when they hold at most its capacity of keys, else in
// place in global memory with the other key buffer as scratch. A pass whose
// digit is the same for every key of the range leaves it as it is and is
// skipped. A stable sort has one result, so this is the order of the
// eight-pass sort.
constexpr int kTopShift = 47;
// Block shapes of the bucket sort: a block of T threads holds up to 5 rounds
// of 64 keys per wave (kCap = 5 T) and starts from tiles of kCap - 1024
// keys, so a range never exceeds kCap when no bucket holds more than 1024
// keys. Large sorts use 1024-thread blocks (4096-key tiles), smaller ones
// 256-thread blocks (256-key tiles), so that both give enough blocks.
template <int T>
struct LocalShape {
    static constexpr int kThreads = T;
    static constexpr int kWaves = T / 64;
    static constexpr int kCap = 5 * T;
    static constexpr int kWaveKeys = kCap / kWaves;  // 5 rounds of 64
    static constexpr int kTile = kCap - 1024;
};
using LocalBig = LocalShape<1024>;
using LocalSmall = LocalShape<256>;
constexpr int kBucketMax = 1024;  // bucket bound both shapes are sized for
// Buckets sorted by comparison instead of radix passes: when the previous
// build held at most kRankPerNode bodies per level-5 node on average (a
// bucket is half such a node), in ranges whose buckets all hold at most
// kRankMax keys. Each key's comparisons walk its bucket in LDS, so the cost
// grows with the bucket; with tens of keys per bucket the passes are faster.
constexpr int kRankMax = 32;
constexpr int64_t kRankPerNode = 8;
static_assert(LocalBig::kTile > 0 && LocalSmall::kTile > 0, "tiles");
constexpr int64_t kBigSortFrom = (int64_t)256 * LocalBig::kTile;  // 256 blocks of the big shape

template <typename Sh>
struct LocalScratch {
    uint32_t whist[Sh::kWaves][256];  // per-wave digit counts, then offsets
    uint32_t base[256];               // where each digit's keys of a chunk start
    uint32_t part[4];                 // wave totals of a 256-entry scan
};

// Exclusive scan of v over threads 0..255 (the first four waves); every
// thread of the block calls it.
__device__ inline uint32_t scan256_excl(uint32_t v, uint32_t *part)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t x = tid < 256 ? v : 0u;
    const uint32_t incl = wave_incl_scan(x);
    if (lane == 63 && wave < 4) part[wave] = incl;
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < 4 && w < wave; w++) add += part[w];
    __syncthreads();  // part is reused by the next call
    return add + incl - x;
}

// One stable counting pass of the block over keys ksrc[0..m) with values
// vsrc into kdst / vdst, on the digit (key >> shift) & 255, in chunks of
// kCap keys taken in order. In a chunk, wave w holds keys w*kWaveKeys .. in
// rounds of 64 and ranks them among equal digits with ballots and a per-wave
// digit count; a key of digit d then goes to base[d] + (keys of d in earlier
// waves) + rank, and base[d] advances by the chunk's count of d. For
// m > kCap, base starts from a count of every digit over all keys.
template <typename Sh, typename KS, typename VS, typename KD, typename VD>
__device__ __forceinline__ void block_radix_pass(KS ksrc, VS vsrc, KD kdst, VD vdst, int64_t m,
                                                 int shift, LocalScratch<Sh> &S)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool multi = m > Sh::kCap;
    if (multi) {
        if (tid < 256) S.base[tid] = 0u;
        __syncthreads();
        for (int64_t i = tid; i < m; i += Sh::kThreads)
            atomicAdd(&S.base[(uint32_t)(ksrc[i] >> shift) & 255u], 1u);
        __syncthreads();
        const uint32_t ex = scan256_excl(tid < 256 ? S.base[tid] : 0u, S.part);
        if (tid < 256) S.base[tid] = ex;
        __syncthreads();
    }
    for (int64_t c0 = 0; c0 < m; c0 += Sh::kCap) {
        const int cm = (int)(m - c0 < Sh::kCap ? m - c0 : Sh::kCap);
        for (int i = tid; i < Sh::kWaves * 256; i += Sh::kThreads) (&S.whist[0][0])[i] = 0u;
        __syncthreads();
        uint32_t rank[Sh::kWaveKeys / 64], dig[Sh::kWaveKeys / 64];
#pragma unroll
        for (int r = 0; r < Sh::kWaveKeys / 64; r++) {
            const int i = wave * Sh::kWaveKeys + r * 64 + lane;
            const bool valid = i < cm;
            const uint32_t d = valid ? (uint32_t)(ksrc[c0 + i] >> shift) & 255u : 0u;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int bt = 0; bt < 8; bt++) {
                const bool bit = (d >> bt) & 1u;
                const uint64_t bal = __ballot(bit);
                peers &= bit ? bal : ~bal;
            }
            const uint64_t lower = peers & lanemask_lt(lane);
            const uint32_t before = valid ? S.whist[wave][d] : 0u;
            if (valid && lower == 0) S.whist[wave][d] = before + (uint32_t)__popcll(peers);
            rank[r] = before + (uint32_t)__popcll(lower);
            dig[r] = d;
        }
        __syncthreads();
        // digit tid: the offsets of the waves and the chunk's total
        uint32_t run = 0;
        if (tid < 256)
            for (int w = 0; w < Sh::kWaves; w++) {
                const uint32_t c = S.whist[w][tid];
                S.whist[w][tid] = run;
                run += c;
            }
        if (!multi) {
            const uint32_t ex = scan256_excl(run, S.part);
            if (tid < 256) S.base[tid] = ex;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < Sh::kWaveKeys / 64; r++) {
            const int i = wave * Sh::kWaveKeys + r * 64 + lane;
            if (i < cm) {
                const uint32_t o = S.base[dig[r]] + S.whist[wave][dig[r]] + rank[r];
                kdst[o] = ksrc[c0 + i];
                vdst[o] = vsrc[c0 + i];
            }
        }
        __syncthreads();
        if (multi && tid < 256) S.base[tid] += run;
        __syncthreads();
    }
}

template <typename Sh>
__global__ __launch_bounds__(Sh::kThreads) void k_sort_local(uint64_t *__restrict__ keys,
                                                             uint32_t *__restrict__ idx,
                                                             uint64_t *__restrict__ ktmp,
                                                             uint32_t *__restrict__ itmp,
                                                             int64_t n, int rank_small,
                                                             const int64_t *__restrict__ offsets,
                                                             int ns)
{
    __shared__ LocalScratch<Sh> S;
    __shared__ uint64_t skey[2][Sh::kCap];
    __shared__ uint32_t sval[2][Sh::kCap];
    __shared__ int64_t srange[2];
    __shared__ uint32_t sdiff[2];
    __shared__ uint32_t sbig;  // a bucket of more than kRankMax keys in the range
    __shared__ int64_t soff[kLdsScenes + 1];  // scene starts in sorted order (several scenes)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t t0 = (int64_t)blockIdx.x * Sh::kTile;
    const int64_t t1 = t0 + Sh::kTile < n ? t0 + Sh::kTile : n;
    // Several scenes (at most kLdsScenes): each keeps its caller range of
    // positions, so a bucket also ends where a scene starts.
    if (ns > 1)
        for (int i = tid; i <= ns; i += Sh::kThreads) soff[i] = offsets[i];
    __syncthreads();
    auto next_start = [&](int64_t x) {  // the first scene start at or after x (n past the last)
        if (ns <= 1) return n;
        int lo = 0, hi = ns;  // soff[hi] = n >= x
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (soff[mid] >= x)
                hi = mid;
            else
                lo = mid + 1;
        }
        return soff[lo];
    };
    // wave 0: the first bucket that starts in [t0, t1) (past the one holding
    // key t0 - 1); wave 1: the end of the bucket holding key t1 - 1. Within a
    // scene buckets are in ascending order of their top bits, so each ends at
    // the first key whose top bits differ from the search start's, or at the
    // next scene's start.
    if (wave < 2) {
        const int64_t from = wave == 0 ? t0 : t1;
        int64_t pos = from;
        if (wave == 1 || t0 > 0) {
            const uint64_t top = keys[wave == 0 ? t0 - 1 : t1 - 1] >> kTopShift;
            for (int64_t c = from;; c += 64) {
                const int64_t i = c + lane;
                const bool differs = i >= n || (keys[i] >> kTopShift) != top;
                const uint64_t bal = __ballot(differs);
                if (bal) {
                    pos = c + __builtin_ctzll(bal);
                    break;
                }
            }
            pos = min(pos, next_start(from));
        }
        if (lane == 0) srange[wave] = pos;
    }
    __syncthreads();
    const int64_t ra = srange[0], rb = srange[1];
    if (ra >= t1) return;  // no bucket starts here: the block of its start sorts it
    // the range [ra, rb) one scene at a time
    auto sort_range = [&](const int64_t a, const int64_t m) {
        __syncthreads();  // the previous range is done with the LDS
        if (tid < 2) sdiff[tid] = 0u;
        __syncthreads();
        // the key bits that differ somewhere in the range (OR of key ^ first key)
        {
            const uint64_t k0 = keys[a];
            uint64_t d = 0;
            for (int64_t i = tid; i < m; i += Sh::kThreads) d |= keys[a + i] ^ k0;
            for (int o = 32; o > 0; o >>= 1) d |= __shfl_xor(d, o);
            if (lane == 0) {
                atomicOr(&sdiff[0], (uint32_t)d);
                atomicOr(&sdiff[1], (uint32_t)(d >> 32));
            }
        }
        __syncthreads();
        const uint64_t diff = (uint64_t)sdiff[1] << 32 | sdiff[0];
        if (m <= Sh::kCap) {
            for (int i = tid; i < m; i += Sh::kThreads) {
                skey[0][i] = keys[a + i];
                sval[0][i] = idx[a + i];
            }
            if (tid == 0) sbig = rank_small ? 0u : 1u;
            __syncthreads();
            // With rank_small, and buckets of at most kRankMax keys: each key's
            // place is its bucket's start plus the number of keys of the bucket
            // before it in (key, position) order, a stable sort by comparison,
            // with no radix passes. A larger bucket sends the whole range to the
            // radix passes below.
            constexpr int kR = Sh::kCap / Sh::kThreads;
            int32_t dest[kR];
#pragma unroll
            for (int r = 0; r < kR; r++) {
                const int i = tid + r * Sh::kThreads;
                dest[r] = -1;
                if (!rank_small || i >= m) continue;
                const uint64_t k = skey[0][i];
                const uint64_t top = k >> kTopShift;
                int bs = i, be = i + 1;
                while (bs > 0 && i - bs < kRankMax && (skey[0][bs - 1] >> kTopShift) == top) bs--;
                while (be < m && be - bs <= kRankMax && (skey[0][be] >> kTopShift) == top) be++;
                const bool big = be - bs > kRankMax ||
                                 (bs > 0 && i - bs == kRankMax && (skey[0][bs - 1] >> kTopShift) == top);
                if (big) {
                    sbig = 1u;
                    continue;
                }
                int32_t rank = bs;
                for (int j = bs; j < be; j++) {
                    const uint64_t kj = skey[0][j];
                    rank += kj < k || (kj == k && j < i);
                }
                dest[r] = rank;
            }
            __syncthreads();
            if (sbig == 0u) {  // the same on every thread
#pragma unroll
                for (int r = 0; r < kR; r++) {
                    const int i = tid + r * Sh::kThreads;
                    if (i < m) {
                        keys[a + dest[r]] = skey[0][i];
                        idx[a + dest[r]] = sval[0][i];
                    }
                }
                return;
            }
            int src = 0;
            for (int pass = 0; pass < 8; pass++) {
                if (((diff >> (8 * pass)) & 255u) == 0) continue;  // the same on every thread
                block_radix_pass<Sh>(skey[src], sval[src], skey[src ^ 1], sval[src ^ 1], m, 8 * pass,
                                     S);
                src ^= 1;
            }
            for (int i = tid; i < m; i += Sh::kThreads) {
                keys[a + i] = skey[src][i];
                idx[a + i] = sval[src][i];
            }
        } else {
            // buffers alternate between the keys and the scratch; an odd number
            // of passes ends with a copy back
            bool in_keys = true;
            for (int pass = 0; pass < 8; pass++) {
                if (((diff >> (8 * pass)) & 255u) == 0) continue;
                if (in_keys)
                    block_radix_pass<Sh>(keys + a, idx + a, ktmp + a, itmp + a, m, 8 * pass, S);
                else
                    block_radix_pass<Sh>(ktmp + a, itmp + a, keys + a, idx + a, m, 8 * pass, S);
                in_keys = !in_keys;
            }
            if (!in_keys) {
                for (int64_t i = tid; i < m; i += Sh::kThreads) {
                    keys[a + i] = ktmp[a + i];
                    idx[a + i] = itmp[a + i];
                }
            }
        }
    };
    for (int64_t sa = ra; sa < rb;) {
        const int64_t sb = min(rb, next_start(sa + 1));
        sort_range(sa, sb - sa);
        sa = sb;
    }
}

#ifdef BHX_CHECKS
// The checked build's verification of a one-scene sort: keys in order and
// every index inside the array.
__global__ __launch_bounds__(256) void k_check_order(const uint64_t *__restrict__ keys,
                                                     const uint32_t *__restrict__ idx, int64_t n,
                                                     const int64_t *__restrict__ offsets, int ns)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    BHX_CHECK(idx[i] < n, CK_INDEX);
    if (i == 0 || keys[i - 1] <= keys[i]) return;
    // a descent is in order only where a scene starts
    bool start = false;
    if (ns > 1) {
        int lo = 0, hi = ns;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (offsets[mid] >= i)
                hi = mid;
            else
                lo = mid + 1;
        }
        start = offsets[lo] == i;
    }
    BHX_CHECK(start, CK_ORDER);
}
#endif

// ------------------------------------------------------------- 4. gather

// With mark: the first sorted body of each non-empty level-kPrefixLevels
// cell, where the cell part of the key changes (one writer per cell), for
// k_prefix_levels.
__device__ inline void prefix_mark(const uint64_t *__restrict__ keys, int64_t s,
                                   int32_t *__restrict__ mark)
{
    const uint32_t c = (uint32_t)(keys[s] >> kPrefixShift);
    if (s == 0 || (uint32_t)(keys[s - 1] >> kPrefixShift) != c) mark[c] = (int32_t)s;
}

__global__ __launch_bounds__(256) void k_gather(const double *__restrict__ pos,
                                                const double *__restrict__ mass,
                                                const double *__restrict__ eps,
                                                const uint32_t *__restrict__ idx, int64_t n,
                                                Body *__restrict__ body,
                                                double *__restrict__ beps2,
                                                const uint64_t *__restrict__ keys,
                                                int32_t *__restrict__ mark)
{
    int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    if (mark) prefix_mark(keys, s, mark);
    uint32_t i = idx[s];
    if (!check_ok(i < n, CK_INDEX)) i = 0;
    body[s] = Body{pos[3 * (int64_t)i], pos[3 * (int64_t)i + 1], pos[3 * (int64_t)i + 2], mass[i]};
    if (eps) {
        double e = eps[i];
        beps2[s] = e * e;
    }
}

// The state of a multi-step call into the new order: idx holds the S index
// of each sorted body on entry and its caller index on return.
__global__ __launch_bounds__(256) void k_gather_state(const Body *__restrict__ sbody,
                                                      const double *__restrict__ svel,
                                                      const double *__restrict__ seps2,
                                                      const uint32_t *__restrict__ scidx,
                                                      int64_t n, uint32_t *__restrict__ idx,
                                                      Body *__restrict__ body,
                                                      double *__restrict__ tvel,
                                                      double *__restrict__ beps2,
                                                      const uint64_t *__restrict__ keys,
                                                      int32_t *__restrict__ mark)
{
    int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    if (mark) prefix_mark(keys, s, mark);
    int64_t p = idx[s];
    if (!check_ok(p < n, CK_INDEX)) p = 0;
    body[s] = sbody[p];
    for (int a = 0; a < 3; a++) tvel[3 * s + a] = svel[3 * p + a];
    if (seps2) beps2[s] = seps2[p];
    idx[s] = scidx[p];
}

// -------------------------------------------------------------- 5. build

// First node and node count of `level`, clamped to the node table: after an
// overflow (flagged ST_CAPACITY) a level counter can exceed what was written.
__device__ inline void level_range(const int32_t *counts, int level, int64_t node_cap,
                                   int32_t *beg, int32_t *cnt)
{
    int64_t b = 0;
    for (int l = 0; l < level; l++) {
        int64_t c = counts[l];
        b += c < node_cap - b ? c : node_cap - b;
    }
    int64_t c = counts[level];
    *beg = (int32_t)b;
    *cnt = (int32_t)(c < node_cap - b ? c : node_cap - b);
}

// Splits every node of `level` holding more than `leaf` bodies, eight lanes
// per node (one chunk: blockDim / 8 nodes): lane o finds the first body of
// octant o, and the non-empty children are written contiguously in octant
// order. A step of the block takes one chunk of nodes; or, `compact` (levels
// where most nodes are leaves), one node per thread, of which the ones that
// split are listed in LDS and split chunk by chunk, so that a leaf costs one
// load. All nodes of a chunk reserve their children with a single atomic on
// the next level's count (scans over the wave and over the block's waves give
// each node its offset): one atomic per node or per wave serialises on that
// counter. Must be called by every thread of the block (a multiple of 64
// threads, at most 1024); every thread runs the same loop iterations.
// `counts` is the per-level node count array: the tree header's, or a copy
// in LDS that a single-block kernel keeps and writes back. The block's steps
// start at nodes b_first + j stride, j = 0, 1, ... (b_first = block index x
// nodes per step; stride = that times the number of blocks).
// Nodes of at most this many bodies find their octant ranges by counting
// (each octant's count fits a byte), larger ones by binary search.
constexpr int32_t kLinearSplit = 64;

template <bool compact>
__device__ inline void build_nodes(int level, const uint64_t *__restrict__ keys, int32_t *counts,
                                   uint32_t *status, int32_t *cell_max,
                                   NodeInfo *__restrict__ ninfo, int64_t node_cap, int leaf,
                                   int64_t b_first, int64_t stride)
{
    __shared__ uint32_t s_wtot[16];
    __shared__ int32_t s_base;
    __shared__ int32_t s_cmax;
    __shared__ int32_t s_list[compact ? 1024 : 1];  // the step's nodes that split
    int32_t beg, cnt;
    level_range(counts, level, node_cap, &beg, &cnt);
    const int32_t next_beg = beg + cnt;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int o = threadIdx.x & 7, gl = lane & ~7;
    const int shift = 60 - 3 * level;  // bits of the child octant at level + 1
    // level kHintLevel: the block's largest node, merged into cell_max once
    int32_t cmax = 0;
    if (level == kHintLevel && threadIdx.x == 0) s_cmax = 0;
    const uint32_t chunk = blockDim.x >> 3;
    for (int64_t b0 = b_first; b0 < cnt; b0 += stride) {
        uint32_t nlist;  // nodes of the step to give eight lanes each
        if constexpr (compact) {
            // one node per thread: list the ones that split
            const int64_t g = b0 + threadIdx.x;
            bool splits = false;
            if (g < cnt) {
                const int32_t c = ninfo[beg + (int32_t)g].count;
                splits = c > leaf && level < kMaxLevel;
                if (level == kHintLevel) cmax = max(cmax, c);
            }
            const uint64_t sb = __ballot(splits);
            if (lane == 0) s_wtot[wave] = (uint32_t)__popcll(sb);
            __syncthreads();
            uint32_t lbefore = 0;
            nlist = 0;
            for (int w = 0; w < nwaves; w++) {
                const uint32_t t = s_wtot[w];
                if (w < wave) lbefore += t;
                nlist += t;
            }
            if (splits) s_list[lbefore + lanes_below(sb)] = beg + (int32_t)g;
            __syncthreads();  // the list is complete and s_wtot free again
        } else {
            nlist = (uint32_t)min((int64_t)chunk, cnt - b0);
        }
        for (uint32_t c0 = 0; c0 < nlist; c0 += chunk) {
            const uint32_t gi = c0 + (threadIdx.x >> 3);
            const bool live = gi < nlist;
            const uint32_t gl_node = live ? gi : c0;
            int32_t k;
            if constexpr (compact)
                k = s_list[gl_node];
            else
                k = beg + (int32_t)(b0 + gl_node);
            const NodeInfo info = ninfo[k];
            if (!compact && level == kHintLevel && live) cmax = max(cmax, info.count);
            const bool split = live && info.count > leaf && level < kMaxLevel;
            int32_t start;
            if (info.count <= kLinearSplit) {
                // few bodies: the 8 lanes read them all (independent loads) and
                // count them per octant, one byte per octant, summed over the
                // group; octant o starts after the bodies of octants below it
                uint64_t hist = 0;
                if (split)
                    for (int32_t j = o; j < info.count; j += 8)
                        hist += 1ull << (8 * (int)((keys[info.first + j] >> shift) & 7ull));
                hist += __shfl_xor(hist, 1, 8);
                hist += __shfl_xor(hist, 2, 8);
                hist += __shfl_xor(hist, 4, 8);
                const uint64_t below = o == 0 ? 0ull : hist & (~0ull >> (64 - 8 * o));
                start = info.first + (split ? (int32_t)((below * 0x0101010101010101ull) >> 56) : 0);
            } else {
                int32_t a = info.first, b = split ? info.first + info.count : info.first;
                while (a < b) {
                    int32_t m = (a + b) >> 1;
                    if ((int)((keys[m] >> shift) & 7ull) < o)
                        a = m + 1;
                    else
                        b = m;
                }
                start = a;
            }
            int32_t end = __shfl_down(start, 1, 8);
            if (o == 7) end = info.first + info.count;
            BHX_CHECK(!split || (start >= info.first && start <= end &&
                                 end <= info.first + info.count),
                      CK_PARTITION);
            const bool nonempty = split && end > start;
            const uint32_t gm = (uint32_t)(__ballot(nonempty) >> gl) & 0xffu;
            const int nch = __popc(gm);
            const int rank = __popc(gm & ((1u << o) - 1u));
            const uint32_t mine = o == 0 ? (uint32_t)nch : 0u;
            const uint32_t incl = wave_incl_scan(mine);
            if (lane == 63) s_wtot[wave] = incl;
            __syncthreads();
            uint32_t before = 0, btot = 0;
            for (int w = 0; w < nwaves; w++) {
                const uint32_t t = s_wtot[w];
                if (w < wave) before += t;
                btot += t;
            }
            if (threadIdx.x == 0 && btot > 0)
                s_base = atomicAdd(&counts[level + 1], (int32_t)btot);
            __syncthreads();
            const int32_t base = btot > 0 ? s_base : 0;
            const int32_t slot =
                base + (int32_t)(before + __shfl(incl, gl) - __shfl(mine, gl));
            __syncthreads();  // s_wtot and s_base are rewritten by the next chunk
            if (!split) continue;
            const int64_t cfirst = (int64_t)next_beg + slot;
            if (cfirst + nch > node_cap) {
                if (o == 0) atomicOr(status, ST_CAPACITY);
                continue;
            }
            const int32_t scene_bits = info.lvl_nch & (int32_t)0xffff0000;
            if (nonempty)
                ninfo[cfirst + rank] = NodeInfo{start, end - start, -1, (level + 1) | scene_bits};
            if (o == 0) {
                ninfo[k].child0 = (int32_t)cfirst;
                ninfo[k].lvl_nch = level | (nch << 8) | scene_bits;
            }
        }
        if constexpr (compact) __syncthreads();  // s_list is rewritten by the next step
    }
    if (level == kHintLevel) {  // the same on every thread
        for (int off = 32; off > 0; off >>= 1) cmax = max(cmax, __shfl_xor(cmax, off));
        __syncthreads();
        if (lane == 0 && cmax > 0) atomicMax(&s_cmax, cmax);
        __syncthreads();
        if (threadIdx.x == 0 && s_cmax > 0) atomicMax(cell_max, s_cmax);
    }
}

template <bool compact>
__global__ __launch_bounds__(1024) void k_build_level(int level, const uint64_t *__restrict__ keys,
                                                      TreeHeader *__restrict__ hdr,
                                                      NodeInfo *__restrict__ ninfo,
                                                      int64_t node_cap, int leaf)
{
    const int64_t per_step = compact ? blockDim.x : blockDim.x >> 3;  // nodes per block step
    build_nodes<compact>(level, keys, hdr->level_count, &hdr->status, &hdr->cell_max, ninfo,
                         node_cap, leaf, (int64_t)blockIdx.x * per_step,
                         (int64_t)gridDim.x * per_step);
}

// Levels from..upto-1 in one block, on a copy of the node counts in LDS
// (no other kernel runs meanwhile); stops at the first empty level.
template <bool compact>
__device__ inline void build_levels_block(int from, int upto, const uint64_t *__restrict__ keys,
                                          TreeHeader *__restrict__ hdr,
                                          NodeInfo *__restrict__ ninfo, int64_t node_cap,
                                          int leaf, int32_t *scnt)
{
    for (int level = from; level < upto; level++) {
        if (scnt[level] == 0) break;
        build_nodes<compact>(level, keys, scnt, &hdr->status, &hdr->cell_max, ninfo, node_cap, leaf,
                             0, compact ? blockDim.x : blockDim.x >> 3);
        __syncthreads();
    }
}

// The top levels of a single scene, from the sorted keys. A level-l cell
// holds the bodies whose keys start with its 3 l bits, a contiguous run of
// the sorted keys, so the first body of every level-kPrefixLevels cell
// gives the body range of every cell on levels 1..kPrefixLevels. A cell is a
// node iff it holds a body and its parent holds more than `leaf` (then every
// ancestor does too and splits), and a node's children are its non-empty
// octants: the nodes the level-by-level split creates, numbered here in
// Morton order within each level, with no searches and no atomics.

// Exclusive prefix sums of K values at once over the 1024 threads of a block,
// with their totals; every thread calls it. s_w: LDS [16][K].
template <int K>
__device__ inline void block_excl_scan_1024(uint32_t (&v)[K], uint32_t (&tot)[K],
                                            uint32_t (*s_w)[K])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl[K];
#pragma unroll
    for (int k = 0; k < K; k++) incl[k] = wave_incl_scan(v[k]);
    if (lane == 63)
        for (int k = 0; k < K; k++) s_w[wave][k] = incl[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; k++) {
        uint32_t before = 0, t = 0;
#pragma unroll
        for (int w = 0; w < 16; w++) {  // independent LDS reads, all in flight
            const uint32_t x = s_w[w][k];
            if (w < wave) before += x;
            t += x;
        }
        v[k] = before + incl[k] - v[k];
        tot[k] = t;
    }
    __syncthreads();  // s_w may be reused
}

// Levels 1..kPrefixLevels of one scene of n > 0 sorted bodies (the root,
// node 0, written by k_box_final): one block of 1024 threads. Reads the marks
// the gather wrote (restoring them to "none"), turns them into the first
// body of every level-5 cell (held in LDS, one pad word after every 32 so
// that a thread's 32 consecutive cells fall in distinct banks), and writes
// the nodes of levels 1..5 (those of level 5 unsplit, for the level-5 split),
// the children of the root and of levels 1..4, and the node counts of levels
// 1..5. Thread t decides level-5 cells 32 t..32 t + 31, level-4 cells
// 4 t..4 t + 3 and cell t of levels 1..3; the level-4 and level-5 nodes are
// then written with consecutive lanes on consecutive cells, so that the
// stores of a wave fall on consecutive nodes.
static_assert(kPrefixLevels == 5 && kPrefixCells == 32 * 1024, "one block, 32 cells a thread");
__device__ inline int prefix_pad(int c) { return c + (c >> 5); }
__global__ __launch_bounds__(1024) void k_prefix_levels(int32_t *__restrict__ mark, int64_t n,
                                                        TreeHeader *__restrict__ hdr,
                                                        NodeInfo *__restrict__ ninfo,
                                                        int64_t node_cap, int leaf)
{
    __shared__ int32_t s_st[kPrefixCells + kPrefixCells / 32 + 1];  // first body per cell, padded
    __shared__ int32_t s_wmin[16];
    __shared__ uint32_t s_w[16][5];
    __shared__ uint32_t s_r2[64], s_r3[512];  // ranks of the level-2 and level-3 cells
    __shared__ uint32_t s_r4[1024], s_m4[1024], s_r5[1024], s_m5[1024];  // per thread
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int32_t nn = (int32_t)n;
    // 1. the marks (all loads in flight at once), restored to "none"
    {
        int32_t mv[kPrefixCells / 1024];
#pragma unroll
        for (int k = 0; k < kPrefixCells / 1024; k++) mv[k] = mark[t + 1024 * k];
#pragma unroll
        for (int k = 0; k < kPrefixCells / 1024; k++) {
            s_st[prefix_pad(t + 1024 * k)] = mv[k];
            mark[t + 1024 * k] = INT32_MAX;
        }
    }
    if (t == 0) s_st[prefix_pad(kPrefixCells)] = nn;
    __syncthreads();
    // 2. first body of every cell = the smallest mark at or after it (n past
    // the last): a suffix minimum over the thread's cells and the threads
    // after. With it, this thread's level-4 cells that hold bodies (nz4) and
    // its level-5 cells that hold bodies under a level-4 cell that splits (m5).
    const int c0 = 32 * t;
    uint32_t nz4 = 0, m5 = 0;
    {
        int32_t st[33];
#pragma unroll
        for (int j = 0; j < 32; j++) st[j] = s_st[prefix_pad(c0 + j)];
        int32_t lm = st[0];
#pragma unroll
        for (int j = 1; j < 32; j++) lm = min(lm, st[j]);
        int32_t x = lm;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_down(x, o);
            if (lane + o < 64) x = min(x, y);
        }
        int32_t carry = __shfl_down(x, 1);
        if (lane == 63) carry = INT32_MAX;
        if (lane == 0) s_wmin[wave] = x;
        __syncthreads();
        carry = min(carry, nn);
#pragma unroll
        for (int w = 0; w < 16; w++)
            if (w > wave) carry = min(carry, s_wmin[w]);
        st[32] = carry;
#pragma unroll
        for (int j = 31; j >= 0; j--) st[j] = min(st[j], st[j + 1]);
        BHX_CHECK(st[0] >= 0, CK_PARTITION);
#pragma unroll
        for (int j = 0; j < 32; j++) s_st[prefix_pad(c0 + j)] = st[j];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int32_t c4 = st[8 * q + 8] - st[8 * q];
            if (c4 > 0) nz4 |= 1u << q;
            if (c4 > leaf)
#pragma unroll
                for (int j = 8 * q; j < 8 * q + 8; j++)
                    if (st[j + 1] > st[j]) m5 |= 1u << j;
        }
    }
    __syncthreads();
    auto S = [&](int c) { return s_st[prefix_pad(c)]; };  // first body of level-5 cell c
    auto cnt = [&](int l, int c) {  // bodies of level-l cell c
        const int sh = 3 * (5 - l);
        return S((c + 1) << sh) - S(c << sh);
    };
    // 3. which cells are nodes, level by level
    const bool e1 = t < 8 && cnt(1, t) > 0 && nn > leaf;
    const bool e2 = t < 64 && cnt(2, t) > 0 && cnt(1, t >> 3) > leaf;
    const bool e3 = t < 512 && cnt(3, t) > 0 && cnt(2, t >> 3) > leaf;
    const uint32_t m4 = cnt(3, t >> 1) > leaf ? nz4 : 0u;  // under a level-3 cell that splits
    uint32_t r[5] = {e1 ? 1u : 0u, e2 ? 1u : 0u, e3 ? 1u : 0u, (uint32_t)__popc(m4),
                     (uint32_t)__popc(m5)};
    uint32_t tot[5];
    block_excl_scan_1024<5>(r, tot, s_w);
    if (t < 64) s_r2[t] = r[1];
    if (t < 512) s_r3[t] = r[2];
    s_r4[t] = r[3];
    s_m4[t] = m4;
    s_r5[t] = r[4];
    s_m5[t] = m5;
    __syncthreads();
    // 4. the nodes: level l starts after the nodes of the levels above
    const int64_t beg1 = 1, beg2 = beg1 + tot[0], beg3 = beg2 + tot[1], beg4 = beg3 + tot[2],
                  beg5 = beg4 + tot[3];
    if (beg5 + tot[4] > node_cap) {
        if (t == 0) atomicOr(&hdr->status, ST_CAPACITY);
        return;  // the same on every thread
    }
    auto nonempty8 = [&](int l, int c) {  // non-empty children of level-l cell c, l <= 4
        int k = 0;
        for (int o = 0; o < 8; o++) k += cnt(l + 1, 8 * c + o) > 0;
        return k;
    };
    if (t == 0) {
        for (int l = 1; l <= 5; l++) hdr->level_count[l] = (int32_t)tot[l - 1];
        if (nn > leaf) {
            ninfo[0].child0 = (int32_t)beg1;
            ninfo[0].lvl_nch = nonempty8(0, 0) << 8;
        }
    }
    // levels 1..3: cell t; its first child's rank is that of the first cell
    // of its eight on the next level
    auto upper = [&](int l, bool exists, uint32_t rank, int64_t beg, int64_t beg_next,
                     const uint32_t *rnext, int rsel) {
        if (!exists) return;
        const int32_t c = cnt(l, t);
        NodeInfo ni{S(t << (3 * (5 - l))), c, -1, l};
        if (c > leaf) {
            ni.child0 = (int32_t)(beg_next + rnext[rsel]);
            ni.lvl_nch = l | (nonempty8(l, t) << 8);
        }
        ninfo[beg + rank] = ni;
    };
    upper(1, e1, r[0], beg1, beg2, s_r2, 8 * t);
    upper(2, e2, r[1], beg2, beg3, s_r3, 8 * t);
    upper(3, e3, r[2], beg3, beg4, s_r4, 2 * t);  // level-4 cell 8 t is thread 2 t's first
    // level 4, cell c4 = 1024 k + t (owner thread c4 / 4)
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int c4 = 1024 * k + t, o = c4 >> 2, q = c4 & 3;
        const uint32_t mo = s_m4[o];
        if (!((mo >> q) & 1u)) continue;
        const int32_t first = S(c4 << 3), c = S((c4 + 1) << 3) - first;
        NodeInfo ni{first, c, -1, 4};
        if (c > leaf) {
            const uint32_t m5o = s_m5[o];  // the owner of its children too
            ni.child0 = (int32_t)(beg5 + s_r5[o] + __popc(m5o & ((1u << (8 * q)) - 1u)));
            ni.lvl_nch = 4 | (__popc((m5o >> (8 * q)) & 0xffu) << 8);
        }
        ninfo[beg4 + s_r4[o] + __popc(mo & ((1u << q) - 1u))] = ni;
    }
    // level 5, cell c = 1024 k + t (owner thread c / 32)
#pragma unroll 4
    for (int k = 0; k < 32; k++) {
        const int c = 1024 * k + t, o = c >> 5, j = c & 31;
        const uint32_t m5o = s_m5[o];
        if (!((m5o >> j) & 1u)) continue;
        const int32_t first = S(c);
        ninfo[beg5 + s_r5[o] + __popc(m5o & ((1u << j) - 1u))] =
            NodeInfo{first, S(c + 1) - first, -1, 5};
    }
}

// ------------------------------------------------------------ 6. moments

// Mass, centre of mass and mass-weighted softening of every node of `level`,
// by eq. (COMinternal): from the children of an internal node, from the
// bodies of a leaf. Products and sums are rounded as written.
__device__ inline void moments_nodes(int level, const int32_t *counts,
                                     const NodeInfo *__restrict__ ninfo,
                                     const Body *__restrict__ body,
                                     const double *__restrict__ beps2,
                                     const uint64_t *__restrict__ keys,
                                     const SceneBox *__restrict__ box, NodeMom *__restrict__ nmom,
                                     double *__restrict__ neps2, double *__restrict__ nquad,
                                     int64_t node_cap, int use_eps, int64_t g_first,
                                     int64_t stride)
{
#pragma clang fp contract(off)
    int32_t beg, cnt;
    level_range(counts, level, node_cap, &beg, &cnt);
    for (int64_t g = g_first; g < cnt; g += stride) {
        const int32_t k = beg + (int32_t)g;
        const NodeInfo info = ninfo[k];
        // sums in member order; each group's loads are all issued before
        // its first addition
        double ms = 0.0, mx = 0.0, my = 0.0, mz = 0.0, me = 0.0;
        if (info.child0 < 0) {
            const int32_t end = info.first + info.count;
            for (int32_t s0 = info.first; s0 < end; s0 += 4) {
                Body b[4];
                double e[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int32_t s = s0 + u < end ? s0 + u : s0;
                    b[u] = body[s];
                    e[u] = use_eps ? beps2[s] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    if (s0 + u >= end) break;
                    ms += b[u].m;
                    mx += b[u].x * b[u].m;
                    my += b[u].y * b[u].m;
                    mz += b[u].z * b[u].m;
                    if (use_eps) me += e[u] * b[u].m;
                }
            }
        } else {
            const int nch = node_nchild(info);
            NodeMom cm[8];
            double e[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int32_t c = info.child0 + (u < nch ? u : 0);
                cm[u] = nmom[c];
                e[u] = use_eps ? neps2[c] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; u++) {
                if (u >= nch) break;
                ms += cm[u].m;
                mx += cm[u].x * cm[u].m;
                my += cm[u].y * cm[u].m;
                mz += cm[u].z * cm[u].m;
                if (use_eps) me += e[u] * cm[u].m;
            }
        }
        NodeMom out;
        double e2 = 0.0;
        if (ms > 0.0) {
            out = NodeMom{mx / ms, my / ms, mz / ms, ms};
            e2 = use_eps ? me / ms : 0.0;
        } else {
            // massless cell: its centre
            const uint64_t key = keys[info.first];
            const SceneBox &b = box[node_scene(info)];
            const int sh = kMaxLevel - level;
            const double s = ldexp(b.L, -level);
            out.x = b.x0[0] + ((double)(compact3(key >> 2) >> sh) + 0.5) * s;
            out.y = b.x0[1] + ((double)(compact3(key >> 1) >> sh) + 0.5) * s;
            out.z = b.x0[2] + ((double)(compact3(key) >> sh) + 0.5) * s;
            out.m = 0.0;
        }
        nmom[k] = out;
        if (use_eps) neps2[k] = e2;
        if (nquad) {
            // traceless quadrupole about the centre of mass: from the bodies
            // of a leaf, from the children by the parallel-axis shift
            double q[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            auto add = [&](double dx, double dy, double dz, double m) {
                const double d2 = dx * dx + dy * dy + dz * dz;
                q[0] += m * (3.0 * dx * dx - d2);
                q[1] += m * (3.0 * dy * dy - d2);
                q[2] += m * (3.0 * dz * dz - d2);
                q[3] += m * 3.0 * dx * dy;
                q[4] += m * 3.0 * dx * dz;
                q[5] += m * 3.0 * dy * dz;
            };
            if (info.child0 < 0) {
                for (int32_t s = info.first; s < info.first + info.count; s++) {
                    const Body b = body[s];
                    add(b.x - out.x, b.y - out.y, b.z - out.z, b.m);
                }
            } else {
                const int nch = node_nchild(info);
                for (int32_t c = info.child0; c < info.child0 + nch; c++) {
                    const NodeMom cm = nmom[c];
                    for (int a = 0; a < 6; a++) q[a] += nquad[6 * (int64_t)c + a];
                    add(cm.x - out.x, cm.y - out.y, cm.z - out.z, cm.m);
                }
            }
            for (int a = 0; a < 6; a++) nquad[6 * (int64_t)k + a] = q[a];
        }
    }
}

// The launch hints of the build just finished, into pinned host memory:
// its deepest non-empty level, its largest level-kHintLevel node and its
// node count per level.
__device__ inline void report_hints(const TreeHeader *__restrict__ hdr, int32_t *out)
{
    int d = 0;
    for (int l = 1; l <= kMaxLevel; l++)
        if (hdr->level_count[l] > 0) d = l;
    out[0] = d;
    out[1] = hdr->cell_max;
    for (int l = 0; l < kLevels; l++) out[2 + l] = hdr->level_count[l];
}

__global__ __launch_bounds__(256) void k_moments_level(
    int level, const TreeHeader *__restrict__ hdr, const NodeInfo *__restrict__ ninfo,
    const Body *__restrict__ body, const double *__restrict__ beps2,
    const uint64_t *__restrict__ keys, const SceneBox *__restrict__ box,
    NodeMom *__restrict__ nmom, double *__restrict__ neps2, double *__restrict__ nquad,
    int64_t node_cap, int use_eps, int32_t *__restrict__ depth_out)
{
    moments_nodes(level, hdr->level_count, ninfo, body, beps2, keys, box, nmom, neps2, nquad,
                  node_cap, use_eps, (int64_t)blockIdx.x * 256 + threadIdx.x,
                  (int64_t)gridDim.x * 256);
    // the root level reports the launch hints for the next build
    if (level == 0 && depth_out && blockIdx.x == 0 && threadIdx.x == 0)
        report_hints(hdr, depth_out);
}

// Levels from-1 down to 0 of a single scene in one block, then the depth
// report of k_moments_level at level 0.
__global__ __launch_bounds__(1024) void k_moments_head(
    int from, const TreeHeader *__restrict__ hdr, const NodeInfo *__restrict__ ninfo,
    const Body *__restrict__ body, const double *__restrict__ beps2,
    const uint64_t *__restrict__ keys, const SceneBox *__restrict__ box,
    NodeMom *__restrict__ nmom, double *__restrict__ neps2, double *__restrict__ nquad,
    int64_t node_cap, int use_eps, int32_t *__restrict__ depth_out)
{
    __shared__ int32_t scnt[kLevels + 1];
    if (threadIdx.x <= kLevels) scnt[threadIdx.x] = hdr->level_count[threadIdx.x];
    __syncthreads();
    for (int level = from - 1; level >= 0; level--) {
        moments_nodes(level, scnt, ninfo, body, beps2, keys, box, nmom, neps2, nquad, node_cap,
                      use_eps,
                      threadIdx.x, 1024);
        __syncthreads();
    }
    if (depth_out && threadIdx.x == 0) report_hints(hdr, depth_out);
}

// The deep levels in one block (they hold few nodes): with `split`, first
// the split of levels to..kMaxLevel-1 (stopping at the first empty level,
// the node counts kept in LDS), then the moments of levels kMaxLevel down
// to `to`.
__global__ __launch_bounds__(1024) void k_moments_tail(
    int to, int split, const uint64_t *__restrict__ keys, TreeHeader *__restrict__ hdr,
    NodeInfo *__restrict__ ninfo, const Body *__restrict__ body,
    const double *__restrict__ beps2, const SceneBox *__restrict__ box,
    NodeMom *__restrict__ nmom, double *__restrict__ neps2, double *__restrict__ nquad,
    int64_t node_cap, int leaf, int use_eps)
{
    __shared__ int32_t scnt[kLevels + 1];
    if (threadIdx.x <= kLevels) scnt[threadIdx.x] = hdr->level_count[threadIdx.x];
    __syncthreads();
    if (split) {  // the same on every thread
        build_levels_block<true>(to, kMaxLevel, keys, hdr, ninfo, node_cap, leaf, scnt);
        __syncthreads();
        if (threadIdx.x <= kLevels) hdr->level_count[threadIdx.x] = scnt[threadIdx.x];
    }
    for (int level = kMaxLevel; level >= to; level--) {
        if (scnt[level] == 0) continue;  // the same on every thread
        moments_nodes(level, scnt, ninfo, body, beps2, keys, box, nmom, neps2, nquad, node_cap,
                      use_eps, threadIdx.x, 1024);
        __syncthreads();
    }
}

// ------------------------------------------------- whole build, small scene

// The whole build of one scene of at most kSmallBuild bodies in one block:
// box and input check, keys, an eight-pass stable radix sort of (key, index)
// held in LDS, gather, every level of the tree and the moments.
// Each stage computes what the multi-launch path computes (the same stable
// order, the same node set and moments); a small scene is bound by launch
// latency, which this removes.
constexpr int kSmallThreads = 1024;

__global__ __launch_bounds__(kSmallThreads) void k_build_small(
    const double *__restrict__ pos, const double *__restrict__ mass,
    const double *__restrict__ eps, int64_t n, int leaf, SceneBox *__restrict__ box,
    TreeHeader *__restrict__ hdr, uint64_t *__restrict__ k0, uint32_t *__restrict__ i0,
    Body *__restrict__ body,
    double *__restrict__ beps2, NodeInfo *__restrict__ ninfo, NodeMom *__restrict__ nmom,
    double *__restrict__ neps2, double *__restrict__ nquad, int64_t node_cap,
    int32_t *__restrict__ depth_out)
{
    constexpr int W = kSmallThreads / 64;
    constexpr int kChunk = kSmallBuild / W;  // keys per wave in the sort (4 rounds of 64)
    static_assert(kChunk % 64 == 0, "whole rounds per wave");
    __shared__ unsigned long long red_lo[3], red_hi[3];
    __shared__ uint32_t base[256];
    __shared__ uint32_t whist[W][256];  // per-wave digit counts, then per-wave digit offsets
    __shared__ uint32_t lds4[4];
    // the keys and indices, sorted in LDS (ping-pong)
    __shared__ uint64_t skey[2][kSmallBuild];
    __shared__ uint32_t sval[2][kSmallBuild];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // 1. box and input check
    if (tid < 3) {
        red_lo[tid] = ~0ull;
        red_hi[tid] = 0ull;
    }
    __shared__ int32_t scnt[kLevels + 1];
    if (tid <= kLevels) scnt[tid] = tid == 0 ? 1 : 0;
    __syncthreads();
    {
        unsigned long long lo[3] = {~0ull, ~0ull, ~0ull}, hi[3] = {0ull, 0ull, 0ull};
        bool bad = false;
        for (int64_t i = tid; i < n; i += kSmallThreads) {
            const double x[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
            const double m = mass[i];
            bad |= !(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]));
            bad |= !(isfinite(m) && m >= 0.0);
            if (eps) {
                const double e = eps[i];
                bad |= !(isfinite(e) && e >= 0.0);
            }
            for (int a = 0; a < 3; a++) {
                const unsigned long long c = order_enc(x[a]);
                lo[a] = c < lo[a] ? c : lo[a];
                hi[a] = c > hi[a] ? c : hi[a];
            }
        }
        if (__ballot(bad) && lane == 0) atomicOr(&hdr->status, ST_NONFINITE);
        for (int a = 0; a < 3; a++) {
            atomicMin(&red_lo[a], lo[a]);
            atomicMax(&red_hi[a], hi[a]);
        }
    }
    __syncthreads();
    if (tid == 0) {
        double lo[3], hi[3];
        for (int a = 0; a < 3; a++) {
            box[0].lo_enc[a] = red_lo[a];
            box[0].hi_enc[a] = red_hi[a];
            lo[a] = order_dec(red_lo[a]);
            hi[a] = order_dec(red_hi[a]);
        }
        root_cube(box[0], lo, hi);
        ninfo[0] = NodeInfo{0, (int32_t)n, -1, 0};
    }
    __syncthreads();

    // 2. keys, in LDS
    for (int64_t i = tid; i < n; i += kSmallThreads) {
        skey[0][i] = morton_key(pos + 3 * i, box[0]);
        sval[0][i] = (uint32_t)i;
    }
    __syncthreads();

    // 3. sort, in LDS: wave w holds keys w*kChunk .. (w+1)*kChunk-1 of the
    // current order and ranks them among equal digits with ballots and a
    // per-wave digit count (tile order = wave, round, lane = input order);
    // scans over the waves and over the digits then place every key.
    for (int pass = 0; pass < 8; pass++) {
        const int shift = 8 * pass, src = pass & 1, dst = src ^ 1;
        for (int i = tid; i < W * 256; i += kSmallThreads) (&whist[0][0])[i] = 0;
        __syncthreads();
        uint32_t rank[kChunk / 64], dig[kChunk / 64];
#pragma unroll
        for (int r = 0; r < kChunk / 64; r++) {
            const int i = wave * kChunk + r * 64 + lane;
            const bool valid = i < n;
            const uint32_t d = valid ? (uint32_t)(skey[src][i] >> shift) & 255u : 0u;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; b++) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bal = __ballot(bit);
                peers &= bit ? bal : ~bal;
            }
            const uint64_t lower = peers & lanemask_lt(lane);
            const uint32_t before = valid ? whist[wave][d] : 0u;
            if (valid && lower == 0) whist[wave][d] = before + (uint32_t)__popcll(peers);
            rank[r] = before + (uint32_t)__popcll(lower);
            dig[r] = d;
        }
        __syncthreads();
        // digit tid (first four waves): offsets of the waves, and the exclusive
        // scan of the digit totals; the barriers are reached by every thread
        {
            uint32_t run = 0;
            if (tid < 256)
                for (int w = 0; w < W; w++) {
                    const uint32_t c = whist[w][tid];
                    whist[w][tid] = run;
                    run += c;
                }
            const uint32_t v = wave_incl_scan(run);
            if (lane == 63 && wave < 4) lds4[wave] = v;
            __syncthreads();
            if (tid < 256) {
                uint32_t add = 0;
                for (int w = 0; w < wave; w++) add += lds4[w];
                base[tid] = add + v - run;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kChunk / 64; r++) {
            const int i = wave * kChunk + r * 64 + lane;
            if (i < n) {
                const uint32_t o = base[dig[r]] + whist[wave][dig[r]] + rank[r];
                skey[dst][o] = skey[src][i];
                sval[dst][o] = sval[src][i];
            }
        }
        __syncthreads();
    }
    // eight passes leave the order in buffer 0; the walk and the tree export
    // read the sorted keys and indices from global memory
    for (int64_t i = tid; i < n; i += kSmallThreads) {
        k0[i] = skey[0][i];
        i0[i] = sval[0][i];
    }
    __syncthreads();

    // 4. gather
    for (int64_t s = tid; s < n; s += kSmallThreads) {
        const uint32_t i = sval[0][s];
        body[s] = Body{pos[3 * (int64_t)i], pos[3 * (int64_t)i + 1], pos[3 * (int64_t)i + 2],
                       mass[i]};
        if (eps) {
            const double e = eps[i];
            beps2[s] = e * e;
        }
    }
    __syncthreads();

    // 5. tree, top-down, with the node counts and the sorted keys in LDS
    build_levels_block<false>(0, kMaxLevel, skey[0], hdr, ninfo, node_cap, leaf, scnt);
    __syncthreads();
    // 6. moments, bottom-up
    for (int level = kMaxLevel; level >= 0; level--) {
        if (scnt[level] == 0) continue;  // the same on every thread
        moments_nodes(level, scnt, ninfo, body, beps2, skey[0], box, nmom, neps2, nquad, node_cap,
                      eps != nullptr, tid, kSmallThreads);
        __syncthreads();
    }
    if (tid <= kLevels) hdr->level_count[tid] = scnt[tid];
    if (depth_out && tid == 0) {
        int d = 0;
        for (int l = 1; l <= kMaxLevel; l++)
            if (scnt[l] > 0) d = l;
        depth_out[0] = d;
        depth_out[1] = -1;  // no sort hint from a one-block build
        for (int l = 0; l < kLevels; l++) depth_out[2 + l] = scnt[l];
    }
}

inline unsigned blocks_for(int64_t items, int per_block, unsigned cap)
{
    int64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    return (unsigned)(b < (int64_t)cap ? b : cap);
}

// Upper bound on the nodes of one level: at most 8^level per scene and at
// most n in all.
inline int64_t level_bound(int level, int64_t n, int scenes)
{
    int64_t b = scenes;
    for (int l = 0; l < level && b < n; l++) b *= 8;
    return b < n ? b : n;
}

// One block per scene fills its body range.
__global__ __launch_bounds__(256) void k_scene_of(const int64_t *__restrict__ offsets,
                                                  uint16_t *__restrict__ scene_of)
{
    const int sc = blockIdx.x;
    for (int64_t i = offsets[sc] + threadIdx.x; i < offsets[sc + 1]; i += 256)
        scene_of[i] = (uint16_t)sc;
}

}  // namespace

hipError_t launch_scene_of(hipStream_t s, const int64_t *offsets, int n_scenes,
                           uint16_t *scene_of)
{
    k_scene_of<<<n_scenes, 256, 0, s>>>(offsets, scene_of);
    return hipGetLastError();
}

namespace {

// Stages 2-3: keys of the bodies (coordinates at pos + stride * i) and the
// sort, leaving the sorted order in idx[0]; returns whether it sorted by
// buckets.
bool enqueue_keys_sort(const Workspace &w, hipStream_t s, const Layout &lay, const double *pos,
                       int stride, bool bucket)
{
    const int64_t n = lay.n;
    const int ns = lay.n_scenes;
    const int nblk = (int)((n + kSortTile - 1) / kSortTile);
    const unsigned nb0 = blocks_for(n, 256, 1u << 30);
    if (bucket) {
        // two passes on the top 16 key bits and, for several scenes, one on
        // the scene index (ending in buffer 0), then the buckets in place
        const int passes = ns > 1 ? 3 : 2;
        const int first = passes & 1;
        if (ns == 1)  // the root cube, the keys and the first pass's digit counts
            k_keys_hist<<<nblk, kSortThreads, 0, s>>>(pos, stride, n, w.box, w.hdr, w.ninfo,
                                                      w.keys[0], w.idx[0], kTopShift,
                                                      w.sort_counts, nblk);
        else
            k_keys<<<nb0, 256, 0, s>>>(pos, stride, n, w.box, lay.scene_of, w.keys[first],
                                       w.idx[first]);
        for (int pass = 0; pass < passes; pass++) {
            const int shift = pass < 2 ? kTopShift + 8 * pass : 64;
            const int src = (pass + first) & 1, dst = src ^ 1;
            if (ns > 1 || pass > 0)
                k_sort_hist<<<nblk, kSortThreads, 0, s>>>(w.keys[src], w.idx[src], lay.scene_of,
                                                          lay.offsets, ns, n, shift, w.sort_counts,
                                                          nblk);
            k_sort_scan<<<256, 256, 0, s>>>(w.sort_counts, w.sort_totals, nblk);
            k_sort_scatter<<<nblk, kSortThreads, 0, s>>>(w.keys[src], w.idx[src], lay.scene_of,
                                                         lay.offsets, ns, w.keys[dst], w.idx[dst],
                                                         n, shift, w.sort_counts, w.sort_totals,
                                                         nblk);
        }
        // small buckets are placed by comparison (the previous build's mean
        // bodies per level-5 node picks it; only speed depends on it)
        const int32_t n5 = ((const volatile int32_t *)w.depth_host)[2 + kHintLevel];
        const int rank_small = n5 > 0 && n <= kRankPerNode * (int64_t)n5 ? 1 : 0;
        if (n >= kBigSortFrom)
            k_sort_local<LocalBig>
                <<<(unsigned)((n + LocalBig::kTile - 1) / LocalBig::kTile), LocalBig::kThreads, 0,
                   s>>>(w.keys[0], w.idx[0], w.keys[1], w.idx[1], n, rank_small, lay.offsets, ns);
        else
            k_sort_local<LocalSmall>
                <<<(unsigned)((n + LocalSmall::kTile - 1) / LocalSmall::kTile),
                   LocalSmall::kThreads, 0, s>>>(w.keys[0], w.idx[0], w.keys[1], w.idx[1], n,
                                                 rank_small, lay.offsets, ns);
#ifdef BHX_CHECKS
        k_check_order<<<nb0, 256, 0, s>>>(w.keys[0], w.idx[0], n, lay.offsets, ns);
#endif
        return true;
    }
    // 8 passes on the Morton key, then (several scenes) one on each byte of
    // the scene index that is not always zero; the keys start in the buffer
    // that makes the last pass write buffer 0.
    const int passes = ns > 256 ? 10 : ns > 1 ? 9 : 8;
    const int first = passes & 1;
    k_keys<<<nb0, 256, 0, s>>>(pos, stride, n, w.box, lay.scene_of, w.keys[first], w.idx[first]);
    for (int pass = 0; pass < passes; pass++) {
        const int shift = pass < 8 ? 8 * pass : 64 + 8 * (pass - 8);
        const int src = (pass + first) & 1, dst = src ^ 1;
        k_sort_hist<<<nblk, kSortThreads, 0, s>>>(w.keys[src], w.idx[src], lay.scene_of,
                                                  lay.offsets, ns, n, shift, w.sort_counts, nblk);
        k_sort_scan<<<256, 256, 0, s>>>(w.sort_counts, w.sort_totals, nblk);
        k_sort_scatter<<<nblk, kSortThreads, 0, s>>>(w.keys[src], w.idx[src], lay.scene_of,
                                                     lay.offsets, ns, w.keys[dst], w.idx[dst], n,
                                                     shift, w.sort_counts, w.sort_totals, nblk);
    }
#ifdef BHX_CHECKS
    k_check_order<<<nb0, 256, 0, s>>>(w.keys[0], w.idx[0], n, lay.offsets, ns);
#endif
    return false;
}

// How a build launches its levels, read once from the previous build's hints:
// levels 0..deep-1 get a launch each (the deeper ones share one block), and
// with `prefix` a single scene's levels 1..kPrefixLevels are read off the
// sorted keys instead (the gather writes the marks k_prefix_levels reads).
struct LevelPlan {
    int deep = kMaxLevel, prev = -1;
    bool prefix = false;
};

LevelPlan plan_levels(const Workspace &w, const Layout &lay)
{
    LevelPlan p;
    if (w.depth_host) {
        p.prev = *(const volatile int32_t *)w.depth_host;
        if (p.prev >= 0 && p.prev + 1 < p.deep) p.deep = p.prev + 1;
    }
    p.prefix = lay.n_scenes == 1 && p.deep > kPrefixLevels && w.prefix_mark != nullptr;
    return p;
}

// Stages 5-6 on the sorted bodies (with the plan the gather was launched with).
void enqueue_levels(const Workspace &w, hipStream_t s, const Layout &lay, int leaf, bool use_eps,
                    const LevelPlan &plan)
{
    const int64_t n = lay.n;
    const int ns = lay.n_scenes;
    // Splitting: levels 0..deep-1 get a launch each, sized by the largest
    // scene; the levels from `deep` down, which the previous build on this
    // workspace left empty but for one level of growth, are handled in one
    // block. Moments: the same, and the top levels of a single scene (levels
    // 0..head-1, at most 585 nodes) in one block too. (Splitting the top
    // levels in one block was measured slower: its binary searches over all
    // bodies run four passes deep there.) The split only affects speed.
    const int deep = plan.deep, prev = plan.prev;
    const volatile int32_t *hint = w.depth_host;
    const int head = ns == 1 ? (deep < 4 ? deep : 4) : 0;
    // one scene: levels 1..kPrefixLevels from the marks of the gather in one
    // block instead of one launch per level (when the previous build went deeper)
    if (plan.prefix)
        k_prefix_levels<<<1, 1024, 0, s>>>(w.prefix_mark, n, w.hdr, w.ninfo, w.node_cap, leaf);
    for (int level = plan.prefix ? kPrefixLevels : 0; level < deep; level++) {
        // a level whose next level held no more nodes in the previous build
        // holds mostly leaves: one thread per node, the splitting ones listed;
        // otherwise eight lanes per node. Levels of many nodes take 1024-thread
        // blocks (fewer reservations on the level counter), small ones 256
        // (more CUs for their searches). The choice only affects speed.
        const bool compact =
            prev >= 0 && level < kMaxLevel && hint[2 + level] > 0 &&
            hint[3 + level] <= hint[2 + level];
        const int64_t threads = level_bound(level, n, ns) * (compact ? 1 : 8);
        const int bs = threads >= 65536 ? 1024 : 256;
        const unsigned g = blocks_for(threads, bs, bs == 1024 ? 1024 : 4096);
        if (compact)
            k_build_level<true>
                <<<g, bs, 0, s>>>(level, w.keys[0], w.hdr, w.ninfo, w.node_cap, leaf);
        else
            k_build_level<false>
                <<<g, bs, 0, s>>>(level, w.keys[0], w.hdr, w.ninfo, w.node_cap, leaf);
    }
    // the levels from `deep` down: their split and their moments in one block
    const int ue = use_eps ? 1 : 0;
    k_moments_tail<<<1, 1024, 0, s>>>(deep, deep < kMaxLevel ? 1 : 0, w.keys[0], w.hdr, w.ninfo,
                                      w.body, w.beps2, w.box, w.nmom, w.neps2, w.nquad,
                                      w.node_cap, leaf, ue);
    for (int level = deep - 1; level >= head; level--) {
        const unsigned g = blocks_for(level_bound(level, n, ns), 256, 4096);
        k_moments_level<<<g, 256, 0, s>>>(level, w.hdr, w.ninfo, w.body, w.beps2, w.keys[0], w.box,
                                          w.nmom, w.neps2, w.nquad, w.node_cap, ue, w.depth_dev);
    }
    if (head > 0)
        k_moments_head<<<1, 1024, 0, s>>>(head, w.hdr, w.ninfo, w.body, w.beps2, w.keys[0], w.box,
                                          w.nmom, w.neps2, w.nquad, w.node_cap, ue, w.depth_dev);
}

__global__ __launch_bounds__(64) void k_merge_status(TreeHeader *__restrict__ slot_hdr, int count,
                                                     uint32_t *__restrict__ status)
{
    for (int k = threadIdx.x; k < count; k += 64) {
        const uint32_t st = slot_hdr[k].status;
        if (st) {
            atomicOr(status, st);
            slot_hdr[k].status = 0u;
        }
    }
}

}  // namespace

BHX_DEFINE_TAKE_CHECKS(tree_take_checks)

Workspace slot_view(const Workspace &w, const TreeSlots &t, int k)
{
    Workspace v = w;
    v.body = t.body + (int64_t)k * t.n;
    v.beps2 = t.beps2 + (int64_t)k * t.n;
    v.idx[0] = t.idx + (int64_t)k * t.n;
    v.keys[0] = t.keys + (int64_t)k * t.n;
    v.ninfo = t.ninfo + (int64_t)k * t.node_cap;
    v.nmom = t.nmom + (int64_t)k * t.node_cap;
    v.neps2 = t.neps2 + (int64_t)k * t.node_cap;
    v.node_cap = t.node_cap;
    v.box = t.box + k;
    v.hdr = t.hdr + k;
    v.max_scenes = 1;
    return v;
}

hipError_t launch_merge_status(hipStream_t s, TreeHeader *slot_hdr, int count, uint32_t *status)
{
    if (count <= 0) return hipSuccess;
    k_merge_status<<<1, 64, 0, s>>>(slot_hdr, count, status);
    return hipGetLastError();
}

bool bucket_sort_hint(const Workspace &w, const Layout &lay)
{
    if (lay.n_scenes > kLdsScenes || lay.n <= kSmallBuild || !w.depth_host) return false;
    // a range is a tile plus at most one bucket, and a bucket lies inside one
    // node of level kHintLevel (its top 16 bits fix the first 5 levels)
    const int cell = ((const volatile int32_t *)w.depth_host)[1];
    return cell >= 0 && cell <= kBucketMax;
}

hipError_t launch_build(const Workspace &w, hipStream_t s, const Layout &lay, const double *pos,
                        const double *mass, const double *eps, int leaf, bool *bucket)
{
    if (bucket) *bucket = false;
    const int64_t n = lay.n;
    const int ns = lay.n_scenes;
    if (ns == 1 && n >= 1 && n <= kSmallBuild) {
        k_build_small<<<1, kSmallThreads, 0, s>>>(pos, mass, eps, n, leaf, w.box, w.hdr, w.keys[0],
                                                  w.idx[0], w.body, w.beps2, w.ninfo, w.nmom,
                                                  w.neps2, w.nquad, w.node_cap, w.depth_dev);
        return hipGetLastError();
    }
    const unsigned sb = (unsigned)((ns + 255) / 256);
    k_box_init<<<sb, 256, 0, s>>>(w.box, ns);
    const int nchunks = lay.chunks ? lay.n_chunks : (int)((n + kBoxChunk - 1) / kBoxChunk);
    if (nchunks > 0)
        k_box_chunk<<<nchunks, kBoxThreads, 0, s>>>(pos, mass, eps, n, lay.chunks, w.box, w.hdr);
    // the sort is chosen once (a host read of the previous build's hint); a
    // single scene's bucket sort finishes the box in its key kernel
    const bool bk = n > 0 && bucket_sort_hint(w, lay);
    if (!(bk && ns == 1)) k_box_final<<<sb, 256, 0, s>>>(w.box, ns, lay.offsets, n, w.hdr, w.ninfo);
    if (n == 0) return hipGetLastError();
    enqueue_keys_sort(w, s, lay, pos, 3, bk);
    if (bucket) *bucket = bk;
    const LevelPlan plan = plan_levels(w, lay);
    k_gather<<<blocks_for(n, 256, 1u << 30), 256, 0, s>>>(pos, mass, eps, w.idx[0], n, w.body,
                                                          w.beps2, w.keys[0],
                                                          plan.prefix ? w.prefix_mark : nullptr);
    enqueue_levels(w, s, lay, leaf, eps != nullptr, plan);
    return hipGetLastError();
}

hipError_t launch_build_state(const Workspace &w, hipStream_t s, const Layout &lay, bool use_eps,
                              int leaf, double dt, bool *bucket)
{
    if (bucket) *bucket = false;
    const int64_t n = lay.n;
    const int ns = lay.n_scenes;
    if (n <= 0) return hipSuccess;
    const unsigned sb = (unsigned)((ns + 255) / 256);
    k_box_init<<<sb, 256, 0, s>>>(w.box, ns);
    const int nchunks = lay.chunks ? lay.n_chunks : (int)((n + kBoxChunk - 1) / kBoxChunk);
    k_state_kick_drift<<<nchunks, kBoxThreads, 0, s>>>(
        w.body, w.tvel, w.tacc, w.beps2, w.idx[0], n, 0.5 * dt, dt, lay.chunks, w.sbody, w.svel,
        use_eps ? w.seps2 : nullptr, w.scidx, w.box, w.hdr);
    const bool bk = bucket_sort_hint(w, lay);  // read once, as in launch_build
    if (!(bk && ns == 1)) k_box_final<<<sb, 256, 0, s>>>(w.box, ns, lay.offsets, n, w.hdr, w.ninfo);
    enqueue_keys_sort(w, s, lay, reinterpret_cast<const double *>(w.sbody), 4, bk);
    if (bucket) *bucket = bk;
    const LevelPlan plan = plan_levels(w, lay);
    k_gather_state<<<blocks_for(n, 256, 1u << 30), 256, 0, s>>>(
        w.sbody, w.svel, use_eps ? w.seps2 : nullptr, w.scidx, n, w.idx[0], w.body, w.tvel,
        w.beps2, w.keys[0], plan.prefix ? w.prefix_mark : nullptr);
    enqueue_levels(w, s, lay, leaf, use_eps, plan);
    return hipGetLastError();
}

}  // namespace bhx
