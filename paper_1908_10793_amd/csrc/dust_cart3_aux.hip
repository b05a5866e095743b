// Instantiations of the predictor-source / dust-density tile kernel on the
// binned layout of the uniform-Cartesian FP32 path, for every tile shape.
#include "dust_cart3_aux.h"

namespace dust {

DUST_C3_AUX_SHAPES()

}  // namespace dust
