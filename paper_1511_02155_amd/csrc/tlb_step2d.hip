// Plain D2Q9 step: one workgroup per (strip, chunk) item of one lattice.
// The sweep itself (tlb_sweep2d.hpp) is shared with the batched kernel.
#include "tlb_step2d.hpp"

namespace tlb {


// Instantiated: three, four and five components (Sec. II.E), both depths.
template <typename T>
hipError_t launch_step2d(const StepArgs<T>& a, int width, int depth, bool mrt, int nc, hipStream_t s)
{
    // states past 4 GiB take the kernels with one buffer descriptor per population array
    if ((int64_t)9 * nc * a.N * (int64_t)sizeof(T) > (int64_t)0xFFFFFF00)
        return launch_step2d_big<T>(a, width, depth, mrt, nc, s);
    dim3 grid(a.nitems);
#define TLB_L2(W, D, M, NC)                                                        \
    if (width == W && depth == D && mrt == M && nc == NC) {                        \
        hipLaunchKernelGGL((k_step2d<T, W, D, M, NC, false>), grid, dim3(W), 0, s, a); \
        return hipGetLastError();                                                  \
    }
#define TLB_L2W(D, M, NC) TLB_L2(64, D, M, NC) TLB_L2(128, D, M, NC) TLB_L2(256, D, M, NC)
    TLB_L2W(0, false, 3)
    TLB_L2W(1, false, 3)
    TLB_L2W(0, true, 3)
    TLB_L2W(1, true, 3)
    TLB_L2W(0, false, 4)
    TLB_L2W(0, true, 4)
    TLB_L2W(0, false, 5)
    TLB_L2W(0, true, 5)
    TLB_L2W(1, false, 4)
    TLB_L2W(1, true, 4)
    TLB_L2W(1, false, 5)
    TLB_L2W(1, true, 5)
#undef TLB_L2W
#undef TLB_L2
    return hipErrorInvalidValue;
}

template hipError_t launch_step2d<float>(const StepArgs<float>&, int, int, bool, int, hipStream_t);
template hipError_t launch_step2d<double>(const StepArgs<double>&, int, int, bool, int, hipStream_t);

}  // namespace tlb
