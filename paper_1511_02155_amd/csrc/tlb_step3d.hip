// D3Q19 step kernels of the ternary model (three components); the kernel is in tlb_step3d.hpp.
#include "tlb_step3d.hpp"

namespace tlb {

template <typename T>
hipError_t launch_step3d(const StepArgs<T>& a, int width, int height, int variant, bool mrt, int nc, hipStream_t s)
{
    if (nc == 3) return launch_step3d_n<T, 3>(a, width, height, variant, mrt, s);
    if (nc == 4) return launch_step3d_n4<T>(a, width, height, variant, mrt, s);
    if (nc == 5) return launch_step3d_n5<T>(a, width, height, variant, mrt, s);
    return hipErrorInvalidValue;
}

template hipError_t launch_step3d<float>(const StepArgs<float>&, int, int, int, bool, int, hipStream_t);
template hipError_t launch_step3d<double>(const StepArgs<double>&, int, int, int, bool, int, hipStream_t);

}  // namespace tlb
