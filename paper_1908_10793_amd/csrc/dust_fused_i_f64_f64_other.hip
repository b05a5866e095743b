// Instantiations of the fused tile step: double storage, double arithmetic (2-D Cartesian, cylindrical and spherical boxes).
#include "dust_fused_kern.h"

namespace dust {

DUST_FUSED_G_DECL(, double, double, GEOM_CART, 2, true)
DUST_FUSED_G_DECL(, double, double, GEOM_CART, 2, false)
DUST_FUSED_G_DECL(, double, double, GEOM_CYL, 3, false)
DUST_FUSED_G_DECL(, double, double, GEOM_SPH, 3, false)

}  // namespace dust
