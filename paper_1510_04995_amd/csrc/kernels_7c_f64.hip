// Kernels of the 7c stencil in double precision (naive step and the
// diamond-row variants listed in instantiate.hpp).
#include "instantiate.hpp"

namespace girih {
void register_kernels_7c_f64(std::vector<KernelEntry>& t) { add_family<Stencil7C, double>(t, ST_7C, DT_F64); }
}  // namespace girih
