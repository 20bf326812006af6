// scan_dense_d.hip -- dense leaf-scan instantiations for padded dimensions 20 24 32
// (compiled with the instruction-level-parallelism scheduler).
#include "scan_inst.h"
namespace bkd {
BKD_SCAN_DENSE_INSTANTIATE(20)
BKD_SCAN_DENSE_INSTANTIATE(24)
BKD_SCAN_DENSE_INSTANTIATE(32)
}  // namespace bkd
