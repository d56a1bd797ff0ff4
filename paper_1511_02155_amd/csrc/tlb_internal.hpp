// Internal interface between the C ABI layer and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tlb_device.hpp"

namespace tlb {

// Arguments of the fused step kernels (passed by value).
template <typename T>
struct StepArgs {
    const T* __restrict__ src;  // state u_t = post-collision populations of step t-1 [3][Q][N]
    T* __restrict__ dst;        // u_{t+1}
    const T* __restrict__ wet;  // [2][3][nx*nz] h_m / (alpha^2 kappa_m), or nullptr
    int nx, ny, nz;
    int walls;
    int64_t N;
    int chunk;    // rows (D2Q9) / planes (D3Q19) swept per workgroup
    int nchunks;  // chunks along the sweep axis
    int ntx, nty; // strips (D2Q9: ntx) / tiles (D3Q19: ntx * nty) across the sweep
    int nitems;   // ntx * nty * nchunks
    int flip;     // D2Q9 strips: 1 reverses the sweep direction of every chunk (alternates per step)
    Phys<acc_t<T>> P;
    Phys<float> Pf;  // the same parameters for kernels whose arithmetic is FP32
};

// Map a hardware workgroup id onto a logical work item so that each XCD
// (workgroups are dispatched round-robin over the 8 XCDs) receives a
// contiguous range of items, which share halo rows through that XCD's L2.
__device__ __forceinline__ int xcd_item(int b, int G)
{
    const int q = G >> 3, r = G & 7;
    const int k = b & 7, j = b >> 3;
    return k * q + (k < r ? k : r) + j;
}

template <typename T>
hipError_t launch_step2d(const StepArgs<T>& a, int width, int hold, bool mrt, int nc, hipStream_t s);
template <typename T>
hipError_t launch_step3d(const StepArgs<T>& a, int width, int height, int variant, bool mrt, int nc, hipStream_t s);
template <typename T>
hipError_t launch_step3d_n4(const StepArgs<T>& a, int width, int height, int variant, bool mrt, hipStream_t s);
template <typename T>
hipError_t launch_step3d_n5(const StepArgs<T>& a, int width, int height, int variant, bool mrt, hipStream_t s);

// Propagation alone in the fused step's pattern and launch shape (tlb_stream.hip).
template <typename T>
hipError_t launch_stream_only(const StepArgs<T>& a, int lattice, int width, int height, int nc, hipStream_t s);

// Auxiliary kernels (tlb_aux.hip).
struct AuxGeom {
    int lattice;  // 0 D2Q9, 1 D3Q19
    int nx, ny, nz, walls;
    int64_t N;
    int nc = 3;   // components (3 .. kMaxComp)
};

// 1 / (alpha^2 kappa_m) per component, for the wetting ghost offsets.
struct WetScale {
    double v[kMaxComp];
};

// Row of a TLB_FIELD_* selector in the field buffer ([nc + 8][N]), or -1.
int field_row(int nc, int which);
// Slots of the conservation check for nc components (see k_diag1).
constexpr int diag_slots(int nc) { return 2 * nc + 5; }

template <typename T, typename TIn>
hipError_t launch_init(const AuxGeom& g, const Phys<acc_t<T>>& P, const TIn* C, const TIn* u, const T* wet,
                       T* state, hipStream_t s);
template <typename T>
hipError_t launch_fields(const AuxGeom& g, const Phys<acc_t<T>>& P, const T* state, const T* wet,
                         T* fields /*[11][N] deviations*/, hipStream_t s);
template <typename T, typename TOut>
hipError_t launch_export_field(const AuxGeom& g, const T* fields, int which, TOut* out, hipStream_t s);
template <typename T, typename TOut>
hipError_t launch_get_pops(const AuxGeom& g, const T* state, int species, TOut* out, hipStream_t s);
template <typename T, typename TIn>
hipError_t launch_set_pops(const AuxGeom& g, const TIn* in, int species, T* state, hipStream_t s);
template <typename T>
hipError_t launch_diag(const AuxGeom& g, const T* state, double* partial, int nblocks, double* out,
                       hipStream_t s);
template <typename T, typename TIn>
hipError_t launch_wet(int n, int nc, const TIn* h, const WetScale& inv, T* wet, hipStream_t s);

hipError_t launch_copy16(const void* src, void* dst, int64_t n16, hipStream_t s);

// Reverse step (tlb_adjoint.hip), D2Q9: one sweep kernel per step.
template <typename T>
struct AdjArgs {
    const T* __restrict__ u;     // u_t [27][N]
    const T* __restrict__ lam1;  // lambda_{t+1} [27][N]
    T* __restrict__ lam0;        // lambda_t [27][N]
    const T* __restrict__ wet;   // [2][3][nx] h_m / (alpha^2 kappa_m), or nullptr
    double* __restrict__ dh;     // [2][3][nx], accumulated
    double* __restrict__ kpart;  // [3][nitems], per work item: accumulated, or written when kassign != 0
    int kassign;                 // nonzero: write the item's kappa partials instead of adding them
    int nx, ny, walls;
    int64_t N;
    int chunk, nchunks, nstrips, nitems;  // strips of (width - 6) output columns
    Phys<acc_t<T>> P;
    Phys<float> Pf;  // the same parameters for FP32 arithmetic
};
template <typename T>
hipError_t launch_adjoint_sweep(const AdjArgs<T>& a, int width, int rows, int hoist, hipStream_t s);
template <typename T>
hipError_t launch_adjoint_seed(const AuxGeom& g, const T* dC, T* lam, hipStream_t s);
hipError_t launch_fill0(double* p, int64_t n, hipStream_t s);
// out[m] += sum of part[m][0 .. n) for m < 3, in a fixed order (one launch)
hipError_t launch_reduce_items(const double* part, int64_t n, double* out, hipStream_t s);
template <typename TIn, typename TOut>
hipError_t launch_convert(const TIn* in, TOut* out, int64_t n, hipStream_t s);

constexpr int kDiagBlocks = 1024;
constexpr int kDiagSlots = diag_slots(kMaxComp);  // the most slots any component count uses

}  // namespace tlb
