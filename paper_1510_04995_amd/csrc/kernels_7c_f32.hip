// Kernels of the 7c stencil in float precision (naive step and the
// diamond-row variants listed in instantiate.hpp).
#include "instantiate.hpp"

namespace girih {
void register_kernels_7c_f32(std::vector<KernelEntry>& t) { add_family<Stencil7C, float>(t, ST_7C, DT_F32); }
}  // namespace girih
