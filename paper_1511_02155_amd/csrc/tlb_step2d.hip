// Plain D2Q9 step: one workgroup per (strip, chunk) item of one lattice.
// The sweep itself (tlb_sweep2d.hpp) is shared with the batched kernel.
#include "tlb_sweep2d.hpp"

namespace tlb {

template <typename T, int W, int DEPTH>
__global__ __launch_bounds__(W) __attribute__((amdgpu_waves_per_eu(step2d_waves<T, DEPTH>())))
void k_step2d(StepArgs<T> A)
{
    __shared__ Sweep2Lds<T, W> S;
    const int item = xcd_item(blockIdx.x, A.nitems);
    const int chunk = item / A.ntx;  // chunk-major: an XCD's range covers whole bands
    const int strip = item - chunk * A.ntx;
    sweep2d<T, W, DEPTH>(A, strip, chunk, S);
}

template <typename T>
hipError_t launch_step2d(const StepArgs<T>& a, int width, int depth, hipStream_t s)
{
    dim3 grid(a.nitems);
#define TLB_L2(W, D)                                                               \
    if (width == W && depth == D) {                                                \
        hipLaunchKernelGGL((k_step2d<T, W, D>), grid, dim3(W), 0, s, a);           \
        return hipGetLastError();                                                  \
    }
    TLB_L2(64, 0)
    TLB_L2(128, 0)
    TLB_L2(256, 0)
    TLB_L2(64, 1)
    TLB_L2(128, 1)
    TLB_L2(256, 1)
#undef TLB_L2
    return hipErrorInvalidValue;
}

template hipError_t launch_step2d<float>(const StepArgs<float>&, int, int, hipStream_t);
template hipError_t launch_step2d<double>(const StepArgs<double>&, int, int, hipStream_t);

}  // namespace tlb
