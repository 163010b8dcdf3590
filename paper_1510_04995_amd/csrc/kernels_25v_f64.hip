// Kernels of the 25v stencil in double precision (naive step and the
// diamond-row variants listed in instantiate.hpp).
#include "instantiate.hpp"

namespace girih {
void register_kernels_25v_f64(std::vector<KernelEntry>& t) { add_family<Stencil25V, double>(t, ST_25V, DT_F64); }
}  // namespace girih
