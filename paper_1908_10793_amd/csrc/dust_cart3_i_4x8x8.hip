// Instantiation of the uniform-Cartesian FP32 tile kernel for 4x8x8 tiles.
#include "dust_cart3_kern.h"

namespace dust {

DUST_C3_SHAPE_DECL(, 4, 8, 8)

}  // namespace dust
