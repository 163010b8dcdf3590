// Kernels of the 7v stencil in double precision (naive step and the
// diamond-row variants listed in instantiate.hpp).
#include "instantiate.hpp"

namespace girih {
void register_kernels_7v_f64(std::vector<KernelEntry>& t) { add_family<Stencil7V, double>(t, ST_7V, DT_F64); }
}  // namespace girih
