// The 16-bit partial-MTTKRP kernels (pm16_body.hpp) instantiated for FP16-stored
// tensors (v_mfma_f32_16x16x32_f16).
#include "pm16_body.hpp"

namespace nncpk {
template const void* pm16_kernel_form<NNCP_F16, false>(int, int, int, int, bool);
template const void* pm16_pack_kernel<NNCP_F16>(bool);
}  // namespace nncpk
