// scan_dense_a.hip -- dense leaf-scan instantiations for padded dimensions 2 3 4 5
// (compiled with the instruction-level-parallelism scheduler).
#include "scan_inst.h"
namespace bkd {
BKD_SCAN_DENSE_INSTANTIATE(2)
BKD_SCAN_DENSE_INSTANTIATE(3)
BKD_SCAN_DENSE_INSTANTIATE(4)
BKD_SCAN_DENSE_INSTANTIATE(5)
}  // namespace bkd
