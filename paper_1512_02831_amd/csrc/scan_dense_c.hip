// scan_dense_c.hip -- dense leaf-scan instantiations for padded dimensions 12 15 16
// (compiled with the instruction-level-parallelism scheduler).
#include "scan_inst.h"
namespace bkd {
BKD_SCAN_DENSE_INSTANTIATE(12)
BKD_SCAN_DENSE_INSTANTIATE(15)
BKD_SCAN_DENSE_INSTANTIATE(16)
}  // namespace bkd
