// scan_b.hip -- leaf-scan instantiations for padded dimensions 6 8 10.
#include "scan_inst.h"
namespace bkd {
BKD_SCAN_DENSE_EXTERN(6)
BKD_SCAN_INSTANTIATE(6)
BKD_SCAN_DENSE_EXTERN(8)
BKD_SCAN_INSTANTIATE(8)
BKD_SCAN_DENSE_EXTERN(10)
BKD_SCAN_INSTANTIATE(10)
}  // namespace bkd
