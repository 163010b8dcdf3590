// Kernels of the 25c stencil in float precision (naive step and the
// diamond-row variants listed in instantiate.hpp).
#include "instantiate.hpp"

namespace girih {
void register_kernels_25c_f32(std::vector<KernelEntry>& t) { add_family<Stencil25C, float>(t, ST_25C, DT_F32); }
}  // namespace girih
