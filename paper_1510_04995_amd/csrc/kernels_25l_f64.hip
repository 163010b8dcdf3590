// Kernels of the second-order-in-time 25-point stencil in double precision.
#include "instantiate.hpp"

namespace girih {
void register_kernels_25l_f64(std::vector<KernelEntry>& t) { add_family<Stencil25L, double>(t, ST_25L, DT_F64); }
}  // namespace girih
