// Kernels of the 27-point box stencil in double precision.
#include "instantiate.hpp"

namespace girih {
void register_kernels_27b_f64(std::vector<KernelEntry>& t) { add_box_family<double>(t, ST_27B, DT_F64); }
}  // namespace girih
