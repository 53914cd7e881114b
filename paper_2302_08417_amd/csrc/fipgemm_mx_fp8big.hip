// The E4M3 256 x 256 tile of the mixed-precision GEMM, in a translation unit
// of its own (its instantiation takes as long to compile as all the other
// forms and tiles together).
#include "fip_mx_impl.h"

namespace fip {

hipError_t launch_mx_fp8_big(const MxLaunchDesc& d, bool pack)
{
    return launch_form<kMxFP8, 256>(d, pack);
}

}  // namespace fip
