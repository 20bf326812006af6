// scan_a.hip -- leaf-scan instantiations for padded dimensions 2 3 4 5.
#include "scan_inst.h"
namespace bkd {
BKD_SCAN_DENSE_EXTERN(2)
BKD_SCAN_INSTANTIATE(2)
BKD_SCAN_DENSE_EXTERN(3)
BKD_SCAN_INSTANTIATE(3)
BKD_SCAN_DENSE_EXTERN(4)
BKD_SCAN_INSTANTIATE(4)
BKD_SCAN_DENSE_EXTERN(5)
BKD_SCAN_INSTANTIATE(5)
}  // namespace bkd
