// Convective sweeps with third-order WENO-Z (section 5.2), plain FP64 form.
#include "convective_launch.hpp"

namespace osbli {
namespace cvl {
template hipError_t launch_convective_s<OSBLI_WENOZ3> OSBLI_CONVECTIVE_SIG;
}  // namespace cvl
}  // namespace osbli
