// Kernels of the second-order-in-time 25-point stencil in single precision.
#include "instantiate.hpp"

namespace girih {
void register_kernels_25l_f32(std::vector<KernelEntry>& t) { add_family<Stencil25L, float>(t, ST_25L, DT_F32); }
}  // namespace girih
