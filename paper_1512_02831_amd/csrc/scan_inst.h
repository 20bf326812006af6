// scan_inst.h -- instantiation of the leaf scan for one padded dimension D over all key capacities.
#pragma once
#include "leaf_scan.h"

// The dense scan's instantiations live in files of their own (scan_dense_*.hip),
// compiled with the instruction-level-parallelism scheduler; the files that
// launch them only declare them.
#define BKD_SCAN_DENSE_EACH(D, X)                                                                   \
    X template __global__ void k_leaf_scan<D, 1>(ScanArgs);                                         \
    X template __global__ void k_leaf_scan<D, 2>(ScanArgs);                                         \
    X template __global__ void k_leaf_scan<D, 4>(ScanArgs);                                         \
    X template __global__ void k_leaf_scan<D, 5>(ScanArgs);                                         \
    X template __global__ void k_leaf_scan<D, 8>(ScanArgs);                                         \
    X template __global__ void k_leaf_scan<D, 10>(ScanArgs);                                        \
    X template __global__ void k_leaf_scan<D, 16>(ScanArgs);                                        \
    X template __global__ void k_leaf_scan<D, 32>(ScanArgs);                                        \
    X template __global__ void k_leaf_scan<D, 64>(ScanArgs);
#define BKD_SCAN_DENSE_EXTERN(D) BKD_SCAN_DENSE_EACH(D, extern)
#define BKD_SCAN_DENSE_INSTANTIATE(D) BKD_SCAN_DENSE_EACH(D, )

#define BKD_SCAN_CASE(D, KK)                                                                        \
    case KK:                                                                                        \
        if (!sparse && a.item_count > 0) k_leaf_scan<D, KK><<<grid, SCAN_THREADS, 0, s>>>(a);      \
        if (sparse == 1 && a.sitem_count > 0) k_leaf_scan_sparse<D, KK><<<sgrid, SCAN_THREADS, 0, s>>>(a); \
        if (sparse == 2 && a.tail_count > 0 && a.tail_wide)                                       \
            k_tail<D, KK, TAIL_THREADS_WIDE><<<(unsigned)a.tail_count, TAIL_THREADS_WIDE, 0, s>>>(a); \
        if (sparse == 2 && a.tail_count > 0 && !a.tail_wide)                                      \
            k_tail<D, KK, TAIL_THREADS><<<(unsigned)a.tail_count, TAIL_THREADS, 0, s>>>(a);       \
        break;

#define BKD_SCAN_INSTANTIATE(D)                                                                     \
    template <> void launch_leaf_scan_d<D>(const ScanArgs &a, int K, int sparse, hipStream_t s)                \
    {                                                                                               \
        unsigned grid = (unsigned)(((int64_t)a.item_count + 7) / 8 * 8);                            \
        unsigned sgrid = (unsigned)(((int64_t)a.sitem_count + 31) / 32 * 8);                        \
        switch (K) {                                                                                \
            BKD_SCAN_CASE(D, 1)                                                                     \
            BKD_SCAN_CASE(D, 2)                                                                     \
            BKD_SCAN_CASE(D, 4)                                                                     \
            BKD_SCAN_CASE(D, 5)                                                                     \
            BKD_SCAN_CASE(D, 8)                                                                     \
            BKD_SCAN_CASE(D, 10)                                                                    \
            BKD_SCAN_CASE(D, 16)                                                                    \
            BKD_SCAN_CASE(D, 32)                                                                    \
            BKD_SCAN_CASE(D, 64)                                                                    \
        default:                                                                                    \
            fail(BKD_EINVAL, "unsupported key capacity");                                           \
        }                                                                                           \
    }
