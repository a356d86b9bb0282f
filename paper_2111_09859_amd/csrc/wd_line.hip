// wd_line.hip -- instantiates the line-tile passes of wd_line.h for one
// value type and one points-per-thread count.  The build compiles this
// file once per variant with WD_LINE_T (float / double), WD_LINE_NP
// (1, 2, 4, 8) and WD_LINE_FN (the launcher's name) defined.
#include "wd_line.h"
#include "wd_kernels.h"

#include <atomic>

#if !defined(WD_LINE_T) || !defined(WD_LINE_NP) || !defined(WD_LINE_FN)
#error "wd_line.hip is built once per variant: define WD_LINE_T, WD_LINE_NP, WD_LINE_FN"
#endif

#define WD_CAT2(a, b) a##b
#define WD_CAT(a, b) WD_CAT2(a, b)

namespace wd {

// Workgroups of this variant's kernel for `kind` that one compute unit holds
// at once (registers and LDS permitting), queried once per kind.
int WD_CAT(WD_LINE_FN, _occ)(int kind)
{
    using T = WD_LINE_T;
    constexpr int NP = WD_LINE_NP;
    static std::atomic<int> cache[16];
    if (kind < 0 || kind >= 16) return 1;
    int v = cache[kind].load(std::memory_order_relaxed);
    if (v > 0) return v;
    const void *f = nullptr;
    switch (kind) {
    case PASS_CART: f = reinterpret_cast<const void *>(&k_cart<T, NP>); break;
    case PASS_D1: f = reinterpret_cast<const void *>(&k_d1<T, NP>); break;
    case PASS_D2: f = reinterpret_cast<const void *>(&k_d2<T, NP, false>); break;
    case PASS_D12: f = reinterpret_cast<const void *>(&k_d2<T, NP, true>); break;
    case PASS_FILTER: f = reinterpret_cast<const void *>(&k_filter<T, NP>); break;
    case PASS_LAD: f = reinterpret_cast<const void *>(&k_lad<T, NP>); break;
    default: break;
    }
    int n = 0;
    if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kThreads, 0) != hipSuccess)
        n = 0;
    v = n < 1 ? 1 : n;
    cache[kind].store(v, std::memory_order_relaxed);
    return v;
}

void WD_LINE_FN(int kind, const GridDev *g, const Item *it, int nitems, int l, int stage,
                int nwg, hipStream_t s)
{
    using T = WD_LINE_T;
    constexpr int NP = WD_LINE_NP;
    const dim3 grid(nwg), block(kThreads);
    switch (kind) {
    case PASS_CART:
        hipLaunchKernelGGL((k_cart<T, NP>), grid, block, 0, s, g, it, nitems, l, stage);
        break;
    case PASS_D1:
        hipLaunchKernelGGL((k_d1<T, NP>), grid, block, 0, s, g, it, nitems, l, stage);
        break;
    case PASS_D2:
        hipLaunchKernelGGL((k_d2<T, NP, false>), grid, block, 0, s, g, it, nitems, l, stage);
        break;
    case PASS_D12:
        hipLaunchKernelGGL((k_d2<T, NP, true>), grid, block, 0, s, g, it, nitems, l, stage);
        break;
    case PASS_FILTER:
        hipLaunchKernelGGL((k_filter<T, NP>), grid, block, 0, s, g, it, nitems, l);
        break;
    case PASS_LAD:
        hipLaunchKernelGGL((k_lad<T, NP>), grid, block, 0, s, g, it, nitems, l, stage);
        break;
    default:
        break;
    }
}

}  // namespace wd
