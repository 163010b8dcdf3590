// Kernels of the 27-point box stencil in single precision.
#include "instantiate.hpp"

namespace girih {
void register_kernels_27b_f32(std::vector<KernelEntry>& t) { add_box_family<float>(t, ST_27B, DT_F32); }
}  // namespace girih
