// The 16-bit partial-MTTKRP kernels (pm16_body.hpp) instantiated for BF16-stored
// tensors (v_mfma_f32_16x16x32_bf16).
#include "pm16_body.hpp"

namespace nncpk {
template const void* pm16_kernel_form<NNCP_BF16, false>(int, int, int, int, bool);
template const void* pm16_pack_kernel<NNCP_BF16>(bool);
}  // namespace nncpk
