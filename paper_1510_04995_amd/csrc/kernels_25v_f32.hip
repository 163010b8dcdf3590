// Kernels of the 25v stencil in float precision (naive step and the
// diamond-row variants listed in instantiate.hpp).
#include "instantiate.hpp"

namespace girih {
void register_kernels_25v_f32(std::vector<KernelEntry>& t) { add_family<Stencil25V, float>(t, ST_25V, DT_F32); }
}  // namespace girih
