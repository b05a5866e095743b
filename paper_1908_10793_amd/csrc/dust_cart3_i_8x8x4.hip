// Instantiation of the uniform-Cartesian FP32 tile kernel for 8x8x4 tiles.
#include "dust_cart3_kern.h"

namespace dust {

DUST_C3_SHAPE_DECL(, 8, 8, 4)

}  // namespace dust
