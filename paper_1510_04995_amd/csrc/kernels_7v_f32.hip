// Kernels of the 7v stencil in float precision (naive step and the
// diamond-row variants listed in instantiate.hpp).
#include "instantiate.hpp"

namespace girih {
void register_kernels_7v_f32(std::vector<KernelEntry>& t) { add_family<Stencil7V, float>(t, ST_7V, DT_F32); }
}  // namespace girih
