// Kernels of the 25c stencil in double precision (naive step and the
// diamond-row variants listed in instantiate.hpp).
#include "instantiate.hpp"

namespace girih {
void register_kernels_25c_f64(std::vector<KernelEntry>& t) { add_family<Stencil25C, double>(t, ST_25C, DT_F64); }
}  // namespace girih
