// Propagation alone: the pull of the fused step (with half-way bounce-back)
// and its store, with no moments, stencils or collision, in the fused step's
// work decomposition and launch shape.  It moves exactly the bytes of a step
// in exactly its access pattern, so its bandwidth is the ceiling that pattern
// allows on the device, the reference the fused step is measured against
// beside the plain copy kernel.
#include "tlb_step2d.hpp"
#include "tlb_step3d.hpp"

namespace tlb {

namespace {

// D2Q9: a strip of W columns over a chunk of rows, swept upwards for even chunks and downwards for odd
// ones (the other way round on steps with A.flip), as in sweep2d; each lane pulls its node's 9 NC
// populations and stores them unchanged.
template <typename T, int W, int NC, bool BIG>
__global__ __launch_bounds__(W) void k_stream2d(StepArgs<T> A)
{
    const int item = xcd_item(blockIdx.x, A.nitems);
    const int chunk = item / A.ntx;
    const int strip = item - chunk * A.ntx;
    const int t = threadIdx.x;
    const int x0 = strip * W;
    if (t >= min(W, A.nx - x0)) return;
    const int x = x0 + t;
    const int y0 = chunk * A.chunk;
    const int y1 = min(y0 + A.chunk, A.ny);
    const int dir = ((chunk ^ A.flip) & 1) ? -1 : 1;
    const StateAddr<T, BIG> src(A.src, A.N, NC), dst(A.dst, A.N, NC);
    const uint32_t vo[3] = {(uint32_t)x * (uint32_t)sizeof(T),
                            (uint32_t)(x == 0 ? A.nx - 1 : x - 1) * (uint32_t)sizeof(T),
                            (uint32_t)(x == A.nx - 1 ? 0 : x + 1) * (uint32_t)sizeof(T)};
    T p[9 * NC];
    for (int k = 0; k < y1 - y0; ++k) {
        const int y = dir > 0 ? y0 + k : y1 - 1 - k;
        pull2d<T, NC, BIG>(A, src, vo, y, p);
        const uint32_t row = (uint32_t)y * (uint32_t)A.nx;
#pragma unroll
        for (int i = 0; i < 9; ++i)
#pragma unroll
            for (int s = 0; s < NC; ++s) bstore<T>(p[9 * s + i], dst.rsrc(9 * s + i), vo[0], dst.soff(9 * s + i, row));
    }
}

// D3Q19: a BX x BY tile of columns over a chunk of z planes, as in k_step3d, without the ring, with the
// store policy k_step3d uses for the same state.
template <typename T, int BX, int BY, int NC, bool NT>
__global__ __launch_bounds__(BX* BY) void k_stream3d(StepArgs<T> A)
{
    constexpr int J = 19 * NC;
    const int item = xcd_item(blockIdx.x, A.nitems);
    const int tile = item / A.nchunks;
    const int chunk = item - tile * A.nchunks;
    const int tyi = tile / A.ntx;
    const int txi = tile - tyi * A.ntx;
    const int x0 = txi * BX, y0 = tyi * BY;
    const int t = threadIdx.x;
    const int tx = t % BX, ty = t / BX;
    if (tx >= min(BX, A.nx - x0) || ty >= min(BY, A.ny - y0)) return;
    const int x = x0 + tx, y = y0 + ty;
    const int z0 = chunk * A.chunk;
    const int z1 = min(z0 + A.chunk, A.nz);
    const int64_t PE = plane3d_elems(A.nx, A.ny, J);
    const uint32_t PBYTES = (uint32_t)(PE * (int64_t)sizeof(T));
    uint32_t col[3][3];
    columns<T, NC>(x, y, A.nx, A.ny, col);
    const bool blo = A.walls && y == 0, bhi = A.walls && y == A.ny - 1;
    const bool wall_tile = A.walls && (y0 <= 1 || y0 + BY >= A.ny - 1);
    T p[J];
    for (int z = z0; z < z1; ++z) {
        const int zm = (z == 0) ? A.nz - 1 : z - 1;
        const int zp = (z == A.nz - 1) ? 0 : z + 1;
        const Rsrc rp[3] = {make_rsrc(A.src + (int64_t)zm * PE, PBYTES), make_rsrc(A.src + (int64_t)z * PE, PBYTES),
                            make_rsrc(A.src + (int64_t)zp * PE, PBYTES)};
        pull3d<T, NC>(rp, col, wall_tile, blo, bhi, p);
        const Rsrc rd = make_rsrc(A.dst + (int64_t)z * PE, PBYTES);
#pragma unroll
        for (int i = 0; i < 19; ++i)
#pragma unroll
            for (int s = 0; s < NC; ++s)
                bstore<T, NT ? kStoreStream : 0>(p[19 * s + i], rd, col[1][1],
                                                 (uint32_t)((19 * s + i) * kBlock3d) * (uint32_t)sizeof(T));
    }
}

}  // namespace

template <typename T>
hipError_t launch_stream_only(const StepArgs<T>& a, int lattice, int width, int height, int nc, hipStream_t s)
{
    const dim3 grid(a.nitems);
    if (lattice == 0) {
        const bool big = (int64_t)9 * nc * a.N * (int64_t)sizeof(T) > (int64_t)0xFFFFFF00;
#define TLB_S2(W, NC)                                                                                   \
    if (width == W && nc == NC) {                                                                       \
        if (big)                                                                                        \
            hipLaunchKernelGGL((k_stream2d<T, W, NC, true>), grid, dim3(W), 0, s, a);                   \
        else                                                                                            \
            hipLaunchKernelGGL((k_stream2d<T, W, NC, false>), grid, dim3(W), 0, s, a);                  \
        return hipGetLastError();                                                                       \
    }
        TLB_S2(64, 3) TLB_S2(128, 3) TLB_S2(256, 3)
        TLB_S2(64, 4) TLB_S2(128, 4) TLB_S2(256, 4)
        TLB_S2(64, 5) TLB_S2(128, 5) TLB_S2(256, 5)
#undef TLB_S2
        return hipErrorInvalidValue;
    }
#define TLB_S3(BX, BY, NC)                                                                         \
    if (width == BX && height == BY && nc == NC) {                                                 \
        if (stream_stores3d<T, NC>(a))                                                             \
            hipLaunchKernelGGL((k_stream3d<T, BX, BY, NC, true>), grid, dim3(BX * BY), 0, s, a);   \
        else                                                                                       \
            hipLaunchKernelGGL((k_stream3d<T, BX, BY, NC, false>), grid, dim3(BX * BY), 0, s, a);  \
        return hipGetLastError();                                                                  \
    }
    TLB_S3(32, 8, 3) TLB_S3(64, 4, 3)
    TLB_S3(32, 8, 4) TLB_S3(64, 4, 4)
    TLB_S3(32, 8, 5) TLB_S3(64, 4, 5)
#undef TLB_S3
    return hipErrorInvalidValue;
}

template hipError_t launch_stream_only<float>(const StepArgs<float>&, int, int, int, int, hipStream_t);
template hipError_t launch_stream_only<double>(const StepArgs<double>&, int, int, int, int, hipStream_t);

}  // namespace tlb
