// Convective sweeps with sixth-order TENO (section 2.5, K = 6), plain FP64 form.
#include "convective_launch.hpp"

namespace osbli {
namespace cvl {
template hipError_t launch_convective_s<OSBLI_TENO6> OSBLI_CONVECTIVE_SIG;
}  // namespace cvl
}  // namespace osbli
