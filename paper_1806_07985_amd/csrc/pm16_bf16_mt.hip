// The 16-bit partial-MTTKRP kernels (pm16_body.hpp) for BF16-stored tensors in
// the form where a work-group streams several M tiles (a separate unit so the
// two forms compile in parallel).
#include "pm16_body.hpp"

namespace nncpk {
template const void* pm16_kernel_form<NNCP_BF16, true>(int, int, int, int, bool);
}  // namespace nncpk
