// Device-side invariant checks of the checked build (compiled with
// BHX_CHECKS, libbhx_checked.so). A failed check sets a bit in a device word
// of its translation unit; bh_sync collects the words and reports any bit as
// BH_E_CHECK. Checks never stop a kernel, so a failing one cannot fault or
// hang the device. In the release build every check compiles to nothing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bhx {

enum : uint32_t {
    CK_STACK = 1u,       // traversal stack beyond its LDS capacity
    CK_RING = 2u,        // interaction queue beyond its ring
    CK_PAIRS = 4u,       // pair list beyond its capacity
    CK_INDEX = 8u,       // a body or node index outside its array
    CK_ORDER = 16u,      // sorted keys out of order
    CK_PARTITION = 32u,  // children that do not partition their parent's bodies
    CK_RANGE = 64u,      // a bucket range beyond what the block holds
};

#ifdef BHX_CHECKS
namespace {
__device__ uint32_t g_check_bits;  // one word per translation unit
}
#define BHX_CHECK(cond, bit)                                          \
    do {                                                              \
        if (!(cond)) atomicOr(&::bhx::g_check_bits, (uint32_t)(bit)); \
    } while (0)
// A check that also guards the access it protects: false (and the bit set)
// when it fails, so the checked build skips the access instead of making it.
__device__ inline bool check_ok(bool ok, uint32_t bit)
{
    if (!ok) atomicOr(&g_check_bits, bit);
    return ok;
}
// Defines `hipError_t name(uint32_t *bits)`: ORs this unit's check word into
// *bits and clears it (host side, synchronous).
#define BHX_DEFINE_TAKE_CHECKS(name)                                                  \
    hipError_t name(uint32_t *bits)                                                   \
    {                                                                                 \
        uint32_t v = 0;                                                               \
        hipError_t e = hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_check_bits), sizeof(v));  \
        if (e != hipSuccess) return e;                                                \
        if (v) {                                                                      \
            const uint32_t zero = 0;                                                  \
            e = hipMemcpyToSymbol(HIP_SYMBOL(g_check_bits), &zero, sizeof(zero));     \
        }                                                                             \
        *bits |= v;                                                                   \
        return e;                                                                     \
    }
#else
#define BHX_CHECK(cond, bit) \
    do {                     \
    } while (0)
__device__ constexpr bool check_ok(bool, uint32_t) { return true; }
#define BHX_DEFINE_TAKE_CHECKS(name) \
    hipError_t name(uint32_t *) { return hipSuccess; }
#endif

// Per translation unit (walk.hip, adjoint.hip, tree.hip).
hipError_t walk_take_checks(uint32_t *bits);
hipError_t adjoint_take_checks(uint32_t *bits);
hipError_t tree_take_checks(uint32_t *bits);

}  // namespace bhx
