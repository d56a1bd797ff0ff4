// Plain D2Q9 step: one workgroup per (strip, chunk) item of one lattice.
// The sweep itself (tlb_sweep2d.hpp) is shared with the batched kernel.
#include "tlb_sweep2d.hpp"

namespace tlb {

template <typename T, int W, int DEPTH, bool MRT>
__global__ __launch_bounds__(W) __attribute__((amdgpu_waves_per_eu(step2d_waves<T, DEPTH>())))
void k_step2d(StepArgs<T> A)
{
    __shared__ Sweep2Lds<T, W> S;
    const int item = xcd_item(blockIdx.x, A.nitems);
    const int chunk = item / A.ntx;  // chunk-major: an XCD's range covers whole bands
    const int strip = item - chunk * A.ntx;
    sweep2d<T, W, DEPTH, MRT>(A, strip, chunk, S);
}

template <typename T>
hipError_t launch_step2d(const StepArgs<T>& a, int width, int depth, bool mrt, hipStream_t s)
{
    dim3 grid(a.nitems);
#define TLB_L2(W, D, M)                                                            \
    if (width == W && depth == D && mrt == M) {                                    \
        hipLaunchKernelGGL((k_step2d<T, W, D, M>), grid, dim3(W), 0, s, a);        \
        return hipGetLastError();                                                  \
    }
    TLB_L2(64, 0, false)
    TLB_L2(128, 0, false)
    TLB_L2(256, 0, false)
    TLB_L2(64, 1, false)
    TLB_L2(128, 1, false)
    TLB_L2(256, 1, false)
    TLB_L2(64, 0, true)
    TLB_L2(128, 0, true)
    TLB_L2(256, 0, true)
    TLB_L2(64, 1, true)
    TLB_L2(128, 1, true)
    TLB_L2(256, 1, true)
#undef TLB_L2
    return hipErrorInvalidValue;
}

template hipError_t launch_step2d<float>(const StepArgs<float>&, int, int, bool, hipStream_t);
template hipError_t launch_step2d<double>(const StepArgs<double>&, int, int, bool, hipStream_t);

}  // namespace tlb
