// scan_dispatch.hip -- choose the leaf-scan instantiation for (d, k).
#include "leaf_scan.h"

namespace bkd {

#define BKD_DECL(D) template <> void launch_leaf_scan_d<D>(const ScanArgs &, int, int, hipStream_t);
BKD_DECL(2) BKD_DECL(3) BKD_DECL(4) BKD_DECL(5) BKD_DECL(6) BKD_DECL(8) BKD_DECL(10) BKD_DECL(12)
BKD_DECL(15) BKD_DECL(16) BKD_DECL(20) BKD_DECL(24) BKD_DECL(32)
#undef BKD_DECL

static const int kDims[] = {2, 3, 4, 5, 6, 8, 10, 12, 15, 16, 20, 24, 32};
static const int kCaps[] = {1, 2, 4, 5, 8, 10, 16, 32, 64};

int padded_dim(int d)
{
    for (int D : kDims)
        if (D >= d) return D;
    return -1;
}

int key_capacity(int k)
{
    for (int K : kCaps)
        if (K >= k) return K;
    return -1;
}

void launch_leaf_scan(const ScanArgs &a, int K, int sparse, hipStream_t s)
{
    if ((sparse == 2 ? a.tail_count : sparse ? a.sitem_count : a.item_count) <= 0) return;
    switch (padded_dim(a.d)) {
    case 2: launch_leaf_scan_d<2>(a, K, sparse, s); break;
    case 3: launch_leaf_scan_d<3>(a, K, sparse, s); break;
    case 4: launch_leaf_scan_d<4>(a, K, sparse, s); break;
    case 5: launch_leaf_scan_d<5>(a, K, sparse, s); break;
    case 6: launch_leaf_scan_d<6>(a, K, sparse, s); break;
    case 8: launch_leaf_scan_d<8>(a, K, sparse, s); break;
    case 10: launch_leaf_scan_d<10>(a, K, sparse, s); break;
    case 12: launch_leaf_scan_d<12>(a, K, sparse, s); break;
    case 15: launch_leaf_scan_d<15>(a, K, sparse, s); break;
    case 16: launch_leaf_scan_d<16>(a, K, sparse, s); break;
    case 20: launch_leaf_scan_d<20>(a, K, sparse, s); break;
    case 24: launch_leaf_scan_d<24>(a, K, sparse, s); break;
    case 32: launch_leaf_scan_d<32>(a, K, sparse, s); break;
    default: fail(BKD_EINVAL, "unsupported dimension");
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(BKD_EDEVICE, std::string("leaf scan launch: ") + hipGetErrorString(e));
}

}  // namespace bkd
