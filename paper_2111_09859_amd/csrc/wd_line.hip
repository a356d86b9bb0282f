// wd_line.hip -- instantiates the line-tile passes of wd_line.h for one
// value type and one points-per-thread count.  The build compiles this
// file once per variant with WD_LINE_T (float / double), WD_LINE_NP
// (1, 2, 4, 8) and WD_LINE_FN (the launcher's name) defined.
#include "wd_line.h"
#include "wd_kernels.h"

#if !defined(WD_LINE_T) || !defined(WD_LINE_NP) || !defined(WD_LINE_FN)
#error "wd_line.hip is built once per variant: define WD_LINE_T, WD_LINE_NP, WD_LINE_FN"
#endif

namespace wd {

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
