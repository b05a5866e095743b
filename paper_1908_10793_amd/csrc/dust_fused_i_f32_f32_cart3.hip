// Instantiations of the fused tile step: float storage, float arithmetic (non-uniform 3-D Cartesian boxes).
#include "dust_fused_kern.h"

namespace dust {

DUST_FUSED_G_DECL(, float, float, GEOM_CART, 3, false)

}  // namespace dust
