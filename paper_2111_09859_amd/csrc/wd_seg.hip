// wd_seg.hip -- launchers of the segmented passes (wd_seg.h), FP32 and FP64,
// segment lengths 16, 24 and 32.
#include "wd_seg.h"
#include "wd_kernels.h"

#include <atomic>

namespace wd {

template <typename T, int M>
static const void *seg_kernel(int kind)
{
    switch (kind) {
    case PASS_SCART: return reinterpret_cast<const void *>(&k_seg_cart<T, M, false>);
    case PASS_SCART_LAST: return reinterpret_cast<const void *>(&k_seg_cart<T, M, true>);
    case PASS_SFILTER: return reinterpret_cast<const void *>(&k_seg_filter<T, M>);
    case PASS_SLAD: return reinterpret_cast<const void *>(&k_seg_lad<T, M>);
    default: return nullptr;
    }
}

static int m_index(int M) { return M == 16 ? 0 : (M == 24 ? 1 : 2); }

template <typename T>
static const void *seg_kernel_m(int kind, int M)
{
    switch (M) {
    case 16: return seg_kernel<T, 16>(kind);
    case 24: return seg_kernel<T, 24>(kind);
    default: return seg_kernel<T, 32>(kind);
    }
}

// one-wave workgroups a compute unit holds by registers alone (LDS is
// accounted for by the caller), queried once per kernel
int seg_blocks_per_cu_regs(int kind, int fp64, int M)
{
    static std::atomic<int> cache[2][4][3];
    const int k = kind == PASS_SCART_LAST ? 3 : kind - PASS_SCART;
    if (k < 0 || k > 3) return 1;
    std::atomic<int> &slot = cache[fp64 ? 1 : 0][k][m_index(M)];
    int v = slot.load(std::memory_order_relaxed);
    if (v > 0) return v;
    const void *f = fp64 ? seg_kernel_m<double>(kind, M) : seg_kernel_m<float>(kind, M);
    int n = 0;
    if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kSegThreads, 0) != hipSuccess)
        n = 0;
    v = n < 1 ? 1 : n;
    slot.store(v, std::memory_order_relaxed);
    return v;
}

template <typename T, int M>
static void seg_launch(int kind, const GridDev *g, const Item *it, int nitems, int l, int stage,
                       int nwg, size_t lds, hipStream_t s)
{
    const dim3 grid(nwg), block(kSegThreads);
    switch (kind) {
    case PASS_SCART:
        hipLaunchKernelGGL((k_seg_cart<T, M, false>), grid, block, lds, s, g, it, nitems, l, stage);
        break;
    case PASS_SCART_LAST:
        hipLaunchKernelGGL((k_seg_cart<T, M, true>), grid, block, lds, s, g, it, nitems, l, stage);
        break;
    case PASS_SFILTER:
        hipLaunchKernelGGL((k_seg_filter<T, M>), grid, block, lds, s, g, it, nitems, l);
        break;
    case PASS_SLAD:
        hipLaunchKernelGGL((k_seg_lad<T, M>), grid, block, lds, s, g, it, nitems, l, stage);
        break;
    default:
        break;
    }
}

template <typename T>
static void seg_launch_m(int kind, int M, const GridDev *g, const Item *it, int nitems, int l,
                         int stage, int nwg, size_t lds, hipStream_t s)
{
    switch (M) {
    case 16: seg_launch<T, 16>(kind, g, it, nitems, l, stage, nwg, lds, s); break;
    case 24: seg_launch<T, 24>(kind, g, it, nitems, l, stage, nwg, lds, s); break;
    default: seg_launch<T, 32>(kind, g, it, nitems, l, stage, nwg, lds, s); break;
    }
}

void launch_seg(int kind, int fp64, int M, const GridDev *g, const Item *it, int nitems, int l,
                int stage, int nwg, size_t lds, hipStream_t s)
{
    if (nitems <= 0) return;
    if (nwg > nitems) nwg = nitems;
    if (fp64) seg_launch_m<double>(kind, M, g, it, nitems, l, stage, nwg, lds, s);
    else seg_launch_m<float>(kind, M, g, it, nitems, l, stage, nwg, lds, s);
}

}  // namespace wd
