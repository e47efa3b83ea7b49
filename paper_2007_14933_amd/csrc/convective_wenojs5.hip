// Convective sweeps with the original WENO weights (section 2.3), plain FP64 form.
#include "convective_launch.hpp"

namespace osbli {
namespace cvl {
template hipError_t launch_convective_s<OSBLI_WENOJS5> OSBLI_CONVECTIVE_SIG;
}  // namespace cvl
}  // namespace osbli
