// scan_dense_b.hip -- dense leaf-scan instantiations for padded dimensions 6 8 10
// (compiled with the instruction-level-parallelism scheduler).
#include "scan_inst.h"
namespace bkd {
BKD_SCAN_DENSE_INSTANTIATE(6)
BKD_SCAN_DENSE_INSTANTIATE(8)
BKD_SCAN_DENSE_INSTANTIATE(10)
}  // namespace bkd
