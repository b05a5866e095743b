// Instantiation of the uniform-Cartesian FP32 tile kernel for 8x4x8 tiles.
#include "dust_cart3_kern.h"

namespace dust {

DUST_C3_SHAPE_DECL(, 8, 4, 8)

}  // namespace dust
