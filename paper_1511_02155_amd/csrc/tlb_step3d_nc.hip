// D3Q19 step kernels of four and five components (Sec. II.E); the kernel is in tlb_step3d.hpp.
#include "tlb_step3d.hpp"

namespace tlb {

template <typename T>
hipError_t launch_step3d_n4(const StepArgs<T>& a, int width, int height, int variant, bool mrt, hipStream_t s)
{
    return launch_step3d_n<T, 4>(a, width, height, variant, mrt, s);
}
template <typename T>
hipError_t launch_step3d_n5(const StepArgs<T>& a, int width, int height, int variant, bool mrt, hipStream_t s)
{
    return launch_step3d_n<T, 5>(a, width, height, variant, mrt, s);
}

template hipError_t launch_step3d_n4<float>(const StepArgs<float>&, int, int, int, bool, hipStream_t);
template hipError_t launch_step3d_n4<double>(const StepArgs<double>&, int, int, int, bool, hipStream_t);
template hipError_t launch_step3d_n5<float>(const StepArgs<float>&, int, int, int, bool, hipStream_t);
template hipError_t launch_step3d_n5<double>(const StepArgs<double>&, int, int, int, bool, hipStream_t);

}  // namespace tlb
