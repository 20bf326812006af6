// scan_d.hip -- leaf-scan instantiations for padded dimensions 20 24 32.
#include "scan_inst.h"
namespace bkd {
BKD_SCAN_DENSE_EXTERN(20)
BKD_SCAN_INSTANTIATE(20)
BKD_SCAN_DENSE_EXTERN(24)
BKD_SCAN_INSTANTIATE(24)
BKD_SCAN_DENSE_EXTERN(32)
BKD_SCAN_INSTANTIATE(32)
}  // namespace bkd
