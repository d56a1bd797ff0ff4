// Plain D2Q9 step kernel: one workgroup per (strip, chunk) item of one lattice.
// The sweep itself (tlb_sweep2d.hpp) is shared with the batched kernel.
#pragma once

#include "tlb_sweep2d.hpp"

namespace tlb {

template <typename T, int W, int DEPTH, bool MRT, int NC, bool BIG>
__global__ __launch_bounds__(W) __attribute__((amdgpu_waves_per_eu(step2d_waves<T, DEPTH>(NC))))
void k_step2d(StepArgs<T> A)
{
    __shared__ Sweep2Lds<T, W, NC> S;
    const int item = xcd_item(blockIdx.x, A.nitems);
    const int chunk = item / A.ntx;  // chunk-major: an XCD's range covers whole bands
    const int strip = item - chunk * A.ntx;
    sweep2d<T, W, DEPTH, MRT, NC, BIG>(A, strip, chunk, S);
}

template <typename T>
hipError_t launch_step2d_big(const StepArgs<T>& a, int width, int depth, bool mrt, int nc, hipStream_t s);

}  // namespace tlb
