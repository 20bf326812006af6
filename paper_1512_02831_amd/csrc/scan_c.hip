// scan_c.hip -- leaf-scan instantiations for padded dimensions 12 15 16.
#include "scan_inst.h"
namespace bkd {
BKD_SCAN_DENSE_EXTERN(12)
BKD_SCAN_INSTANTIATE(12)
BKD_SCAN_DENSE_EXTERN(15)
BKD_SCAN_INSTANTIATE(15)
BKD_SCAN_DENSE_EXTERN(16)
BKD_SCAN_INSTANTIATE(16)
}  // namespace bkd
