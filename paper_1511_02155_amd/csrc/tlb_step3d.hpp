// Fused D3Q19 LB step for gfx950 (same stages as the D2Q9 kernel), for NC = 3
// (the ternary model) to 5 components (Sec. II.E).
//
// Work decomposition.  A workgroup of BX x BY lanes owns a BX x BY tile of
// (x, y) columns and sweeps `chunk` z-planes.  Each lane keeps its own
// column's dC_m for planes z-1, z, z+1 in registers; in-plane neighbours come
// from a double-buffered LDS plane of (BX+2) x (BY+2) entries whose one-node
// ring is filled by the first 2(BX+BY)+4 lanes in an extra pull.  Ghost
// entries beyond a y wall are the adjacent fluid node plus h_m/(alpha^2
// kappa_m).  Per plane and component a lane derives from LDS
//   A  = sum of the 4 in-plane axis neighbours,  Dx, Dy = axis differences,
//   E  = sum of the 4 in-plane diagonals,
//   Fx = sum over y+-1 of [C(x+1) - C(x-1)],  Fy = sum over x+-1 of [C(y+1) - C(y-1)],
// and the D3Q19 isotropic stencils become
//   d_x C = Dx_z/6 + (Fx_z + Dx_{z-1} + Dx_{z+1})/12      (d_y likewise)
//   d_z C = (C_{z+1} - C_{z-1})/6 + (A_{z+1} - A_{z-1})/12
//   lap C = (A_z + C_{z-1} + C_{z+1})/3 + (E_z + A_{z-1} + A_{z+1})/6 - 4 C_z.
// HBM traffic per node and step: 19 NC values read + 19 NC written (NC
// components: 57 + 57 for the ternary model); the ring and the chunk-end
// planes are re-read from L2.  The state is stored in
// plane-major blocks of 64 nodes (tlb_device.hpp), one buffer descriptor per
// z plane.
#pragma once

#include "tlb_internal.hpp"

namespace tlb {

using L19 = D3Q19;

// Pull of node (x, y, z) through buffer accesses.  The state is stored in
// plane-major blocks of 64 nodes (tlb_device.hpp); rp[0..2] are the buffer
// descriptors of planes z-1, z, z+1 (periodic), col[dy + 1][dx + 1] the
// per-lane byte offset of in-plane column (x + dx, y + dy) within a plane,
// and population j = s*19 + i sits j*64 values further (wavefront-uniform),
// so direction i reads col[1 - e_y][1 - e_x] in plane z - e_z.  Where r - e_i
// lies beyond a y wall the lane reads opp(i) at its own node instead
// (half-way bounce-back); only lanes on a wall row of a tile touching a wall
// (wall_tile) take that branch.
template <typename T, int NC>
__device__ __forceinline__ void pull3d(const Rsrc (&rp)[3], const uint32_t (&col)[3][3], bool wall_tile, bool blo,
                                       bool bhi, T* p)
{
    constexpr uint32_t ES = sizeof(T);
#pragma unroll
    for (int s = 0; s < NC; ++s) {
        T* out = p + 19 * s;
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const int ex = L19::ex[i], ey = L19::ey[i], ez = L19::ez[i];
            out[i] = bload<T>(rp[1 - ez], col[1 - ey][1 - ex], (uint32_t)((s * 19 + i) * kBlock3d) * ES);
        }
        if (wall_tile) {
#pragma unroll
            for (int i = 0; i < 19; ++i) {
                const int ey = L19::ey[i];
                if (ey == 0) continue;
                if ((ey == 1 && blo) || (ey == -1 && bhi))
                    out[i] = bload<T>(rp[1], col[1][1], (uint32_t)((s * 19 + L19::opp[i]) * kBlock3d) * ES);
            }
        }
    }
}

// Byte offsets within a plane of the nine in-plane columns around (x, y), periodic in x and y.
template <typename T, int NC>
__device__ __forceinline__ void columns(int x, int y, int nx, int ny, uint32_t (&col)[3][3])
{
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
        int yy = y + dy;
        yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            int xx = x + dx;
            xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
            const uint32_t m = (uint32_t)xx + (uint32_t)nx * (uint32_t)yy;
            col[dy + 1][dx + 1] = (uint32_t)plane3d_index(m, 19 * NC, 0) * (uint32_t)sizeof(T);
        }
    }
}

template <typename T, int NC>
struct PlaneLite {
    T c[NC], A[NC], Dx[NC], Dy[NC];
};
template <typename T, int NC>
struct PlaneFull {
    T c[NC], A[NC], Dx[NC], Dy[NC], E[NC], Fx[NC], Fy[NC];
};

// VAR 0 pulls plane z again (from cache) when it is collided; VAR 1 keeps
// the pulled populations of plane z+1 in registers instead.  VAR 2 also
// pipelines the sweep: the loads of plane z+2 (own column and ring node) are
// issued before plane z is collided and reduced after it, so that their
// latency overlaps the collision, and the populations of plane z+1 wait in
// registers for its collision.  With FP32 storage VAR 0 holds two wavefronts
// per SIMD (about 190 registers), VAR 1 and VAR 2 one (about 260 and 380);
// VAR 2 is built for FP32 storage of three or four components (about 460
// registers at four; five would spill).
// Arithmetic type of the D3Q19 step: the storage type.
template <typename T>
__device__ __forceinline__ const Phys<T>& phys3d(const StepArgs<T>& A);
template <>
__device__ __forceinline__ const Phys<float>& phys3d<float>(const StepArgs<float>& A)
{
    return A.Pf;
}
template <>
__device__ __forceinline__ const Phys<double>& phys3d<double>(const StepArgs<double>& A)
{
    return A.P;
}

template <typename T, int BX, int BY, int VAR, bool MRT, int NC, bool NT>
__global__ __launch_bounds__(BX* BY) void k_step3d(StepArgs<T> A)
{
    using C = T;
    constexpr int J = 19 * NC;  // populations per node
    const Phys<C>& PH = phys3d<T>(A);
    constexpr bool HOLD = VAR == 1;
    __shared__ C lds[2][NC][BY + 2][BX + 2];

    const int item = xcd_item(blockIdx.x, A.nitems);
    const int tile = item / A.nchunks;
    const int chunk = item - tile * A.nchunks;
    const int tyi = tile / A.ntx;
    const int txi = tile - tyi * A.ntx;
    const int x0 = txi * BX, y0 = tyi * BY;
    const int ax = min(BX, A.nx - x0), ay = min(BY, A.ny - y0);
    const int t = threadIdx.x;
    const int tx = t % BX, ty = t / BX;
    const bool active = tx < ax && ty < ay;
    const int x = x0 + min(tx, ax - 1);
    const int y = y0 + min(ty, ay - 1);
    const int z0 = chunk * A.chunk;
    const int z1 = min(z0 + A.chunk, A.nz);

    // Ring node handled by this lane (if any), in tile coordinates.
    const int nh = 2 * (ax + 2) + 2 * ay;
    const bool ring = t < nh;
    int hx, hy;
    if (t < ax + 2) {
        hy = -1;
        hx = t - 1;
    } else if (t < 2 * (ax + 2)) {
        hy = ay;
        hx = t - (ax + 2) - 1;
    } else {
        const int j = t - 2 * (ax + 2);
        hx = (j & 1) ? ax : -1;
        hy = j >> 1;
    }
    int gx = x0 + hx;
    gx = gx < 0 ? gx + A.nx : (gx >= A.nx ? gx - A.nx : gx);
    int gy = y0 + hy;
    int gwall = -1;  // ghost of wall 0 / 1, or -1 for a fluid node
    if (A.walls) {
        if (gy < 0) {
            gwall = 0;
            gy = 0;
        } else if (gy >= A.ny) {
            gwall = 1;
            gy = A.ny - 1;
        }
    } else {
        gy = gy < 0 ? gy + A.ny : (gy >= A.ny ? gy - A.ny : gy);
    }
    const uint32_t nxz = (uint32_t)A.nx * A.nz;

    // one buffer descriptor per z plane (the three source planes of a pull, the destination plane)
    const int64_t PE = plane3d_elems(A.nx, A.ny, J);
    const uint32_t PBYTES = (uint32_t)(PE * (int64_t)sizeof(T));
    auto src_planes = [&](int z, Rsrc (&rp)[3]) {
        const int zm = (z == 0) ? A.nz - 1 : z - 1;
        const int zp = (z == A.nz - 1) ? 0 : z + 1;
        rp[0] = make_rsrc(A.src + (int64_t)zm * PE, PBYTES);
        rp[1] = make_rsrc(A.src + (int64_t)z * PE, PBYTES);
        rp[2] = make_rsrc(A.src + (int64_t)zp * PE, PBYTES);
    };
    auto dst_plane = [&](int z) { return make_rsrc(A.dst + (int64_t)z * PE, PBYTES); };
    uint32_t col[3][3], hcol[3][3];
    columns<T, NC>(x, y, A.nx, A.ny, col);
    columns<T, NC>(gx, gy, A.nx, A.ny, hcol);
    // a tile touches a wall when its rows or its ring rows (y0 - 1 .. y0 + ay) include y = 0 or y = ny - 1
    const bool wall_tile = A.walls && (y0 <= 1 || y0 + ay >= A.ny - 1);
    const bool blo = A.walls && y == 0, bhi = A.walls && y == A.ny - 1;
    const bool hblo = A.walls && gy == 0, hbhi = A.walls && gy == A.ny - 1;

    T fb[J];  // HOLD: populations of plane z
    T fc[J];  // pull buffer (plane z + 1)
    PlaneLite<C, NC> pa;
    PlaneFull<C, NC> pb, pc;
    int buf = 0;

    auto plane = [&](int z, PlaneFull<C, NC>& p) {
        Rsrc rp[3];
        src_planes(z, rp);
        pull3d<T, NC>(rp, col, wall_tile, blo, bhi, fc);
        const Moments<C, NC> mo = moments_as<C, L19, NC>(fc, fc + 19, fc + 38);
        conc_dev<C, NC>(mo, p.c);
        if (active) {
#pragma unroll
            for (int m = 0; m < NC; ++m) lds[buf][m][ty + 1][tx + 1] = p.c[m];
        }
        if (ring) {
            T hf[J];
            pull3d<T, NC>(rp, hcol, wall_tile, hblo, hbhi, hf);
            Moments<C, NC> hm = moments_as<C, L19, NC>(hf, hf + 19, hf + 38);
            C hc[NC];
            conc_dev<C, NC>(hm, hc);
            if (gwall >= 0) {
                const T* __restrict__ wt = A.wet + (size_t)gwall * NC * nxz + gx + (uint32_t)A.nx * z;
#pragma unroll
                for (int m = 0; m < NC; ++m) hc[m] += C(wt[m * nxz]);
            }
#pragma unroll
            for (int m = 0; m < NC; ++m) lds[buf][m][hy + 1][hx + 1] = hc[m];
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            const C l = lds[buf][m][ty + 1][tx];
            const C r = lds[buf][m][ty + 1][tx + 2];
            const C d = lds[buf][m][ty][tx + 1];
            const C u = lds[buf][m][ty + 2][tx + 1];
            const C ld = lds[buf][m][ty][tx];
            const C rd = lds[buf][m][ty][tx + 2];
            const C lu = lds[buf][m][ty + 2][tx];
            const C ru = lds[buf][m][ty + 2][tx + 2];
            p.A[m] = (l + r) + (d + u);
            p.Dx[m] = r - l;
            p.Dy[m] = u - d;
            p.E[m] = (ld + rd) + (lu + ru);
            p.Fx[m] = (rd + ru) - (ld + lu);
            p.Fy[m] = (lu + ru) - (ld + rd);
        }
        buf ^= 1;
    };

    // VAR 2: the loads of plane z (own column, and the ring node on ring lanes)
    // into fc and rf, and their reduction to C_m and plane sums
    // later (the same operations in the same order as plane()).  plane() keeps
    // its own copy of the reduction: issuing the ring pull before the own
    // column's moments, as issue() does, costs variants 0 and 1 about 60 more
    // registers.
    T rf[J];
    auto issue = [&](int z) {
        Rsrc rp[3];
        src_planes(z, rp);
        pull3d<T, NC>(rp, col, wall_tile, blo, bhi, fc);
        if (ring) pull3d<T, NC>(rp, hcol, wall_tile, hblo, hbhi, rf);
    };
    auto finish = [&](int z, PlaneFull<C, NC>& p) {
        const Moments<C, NC> mo = moments_as<C, L19, NC>(fc, fc + 19, fc + 38);
        conc_dev<C, NC>(mo, p.c);
        if (active) {
#pragma unroll
            for (int m = 0; m < NC; ++m) lds[buf][m][ty + 1][tx + 1] = p.c[m];
        }
        if (ring) {
            Moments<C, NC> hm = moments_as<C, L19, NC>(rf, rf + 19, rf + 38);
            C hc[NC];
            conc_dev<C, NC>(hm, hc);
            if (gwall >= 0) {
                const T* __restrict__ wt = A.wet + (size_t)gwall * NC * nxz + gx + (uint32_t)A.nx * z;
#pragma unroll
                for (int m = 0; m < NC; ++m) hc[m] += C(wt[m * nxz]);
            }
#pragma unroll
            for (int m = 0; m < NC; ++m) lds[buf][m][hy + 1][hx + 1] = hc[m];
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            const C l = lds[buf][m][ty + 1][tx];
            const C r = lds[buf][m][ty + 1][tx + 2];
            const C d = lds[buf][m][ty][tx + 1];
            const C u = lds[buf][m][ty + 2][tx + 1];
            const C ld = lds[buf][m][ty][tx];
            const C rd = lds[buf][m][ty][tx + 2];
            const C lu = lds[buf][m][ty + 2][tx];
            const C ru = lds[buf][m][ty + 2][tx + 2];
            p.A[m] = (l + r) + (d + u);
            p.Dx[m] = r - l;
            p.Dy[m] = u - d;
            p.E[m] = (ld + rd) + (lu + ru);
            p.Fx[m] = (rd + ru) - (ld + lu);
            p.Fy[m] = (lu + ru) - (ld + rd);
        }
        buf ^= 1;
    };
    auto wrapz = [&](int z) { return z >= A.nz ? z - A.nz : z; };

    auto hold = [&]() {
        if constexpr (HOLD) {
#pragma unroll
            for (int j = 0; j < J; ++j) fb[j] = fc[j];
        }
    };

    if constexpr (VAR == 2) {
        T fh[J];  // populations of plane z+1, kept for its collision
        // Prologue: planes z0 - 1 and z0 summed, the loads of z0 + 1 issued.
        const int za = (z0 == 0) ? A.nz - 1 : z0 - 1;
        issue(za);
        finish(za, pc);
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            pa.c[m] = pc.c[m];
            pa.A[m] = pc.A[m];
            pa.Dx[m] = pc.Dx[m];
            pa.Dy[m] = pc.Dy[m];
        }
        issue(z0);
        finish(z0, pb);
#pragma unroll
        for (int j = 0; j < J; ++j) fb[j] = fc[j];
        issue(wrapz(z0 + 1));
        for (int z = z0; z < z1; ++z) {
            finish(wrapz(z + 1), pc);
#pragma unroll
            for (int j = 0; j < J; ++j) fh[j] = fc[j];
            if (z + 2 <= z1) issue(wrapz(z + 2));
            C gC[NC][3], lC[NC];
#pragma unroll
            for (int m = 0; m < NC; ++m) {
                gC[m][0] = pb.Dx[m] * C(1.0 / 6.0) + (pb.Fx[m] + pa.Dx[m] + pc.Dx[m]) * C(1.0 / 12.0);
                gC[m][1] = pb.Dy[m] * C(1.0 / 6.0) + (pb.Fy[m] + pa.Dy[m] + pc.Dy[m]) * C(1.0 / 12.0);
                gC[m][2] = (pc.c[m] - pa.c[m]) * C(1.0 / 6.0) + (pc.A[m] - pa.A[m]) * C(1.0 / 12.0);
                lC[m] = (pb.A[m] + pa.c[m] + pc.c[m]) * C(1.0 / 3.0) +
                        (pb.E[m] + pa.A[m] + pc.A[m]) * C(1.0 / 6.0) - pb.c[m] * C(4);
            }
            const Moments<C, NC> mb = moments_as<C, L19, NC>(fb, fb + 19, fb + 38);
            collide<L19, MRT, NC>(PH, mb, pb.c, gC, lC, fb, fb + 19, fb + 38);
            if (active) {
                const Rsrc rd = dst_plane(z);
#pragma unroll
                for (int i = 0; i < 19; ++i)
#pragma unroll
                    for (int s = 0; s < NC; ++s)
                        bstore<T, NT ? kStoreStream : 0>(fb[19 * s + i], rd, col[1][1],
                                                     (uint32_t)((19 * s + i) * kBlock3d) * (uint32_t)sizeof(T));
            }
#pragma unroll
            for (int m = 0; m < NC; ++m) {
                pa.c[m] = pb.c[m];
                pa.A[m] = pb.A[m];
                pa.Dx[m] = pb.Dx[m];
                pa.Dy[m] = pb.Dy[m];
            }
            pb = pc;
#pragma unroll
            for (int j = 0; j < J; ++j) fb[j] = fh[j];
        }
        return;
    }

    // Prologue: planes z0 - 1 and z0.
    {
        const int za = (z0 == 0) ? A.nz - 1 : z0 - 1;
        plane(za, pc);
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            pa.c[m] = pc.c[m];
            pa.A[m] = pc.A[m];
            pa.Dx[m] = pc.Dx[m];
            pa.Dy[m] = pc.Dy[m];
        }
        plane(z0, pb);
        hold();
    }

    for (int z = z0; z < z1; ++z) {
        const int zn = (z + 1 == A.nz) ? 0 : z + 1;
        plane(zn, pc);

        C gC[NC][3], lC[NC];
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            gC[m][0] = pb.Dx[m] * C(1.0 / 6.0) + (pb.Fx[m] + pa.Dx[m] + pc.Dx[m]) * C(1.0 / 12.0);
            gC[m][1] = pb.Dy[m] * C(1.0 / 6.0) + (pb.Fy[m] + pa.Dy[m] + pc.Dy[m]) * C(1.0 / 12.0);
            gC[m][2] = (pc.c[m] - pa.c[m]) * C(1.0 / 6.0) + (pc.A[m] - pa.A[m]) * C(1.0 / 12.0);
            lC[m] = (pb.A[m] + pa.c[m] + pc.c[m]) * C(1.0 / 3.0) + (pb.E[m] + pa.A[m] + pc.A[m]) * C(1.0 / 6.0) -
                    pb.c[m] * C(4);
        }
        if constexpr (!HOLD) {
            Rsrc rp[3];
            src_planes(z, rp);
            pull3d<T, NC>(rp, col, wall_tile, blo, bhi, fb);
        }
        const Moments<C, NC> mb = moments_as<C, L19, NC>(fb, fb + 19, fb + 38);
        collide<L19, MRT, NC>(PH, mb, pb.c, gC, lC, fb, fb + 19, fb + 38);

        if (active) {
            const Rsrc rd = dst_plane(z);
#pragma unroll
            for (int i = 0; i < 19; ++i)
#pragma unroll
                for (int s = 0; s < NC; ++s)
                    bstore<T, NT ? kStoreStream : 0>(fb[19 * s + i], rd, col[1][1],
                                                     (uint32_t)((19 * s + i) * kBlock3d) * (uint32_t)sizeof(T));
        }

#pragma unroll
        for (int m = 0; m < NC; ++m) {
            pa.c[m] = pb.c[m];
            pa.A[m] = pb.A[m];
            pa.Dx[m] = pb.Dx[m];
            pa.Dy[m] = pb.Dy[m];
        }
        pb = pc;
        hold();
    }
}

// Whether a D3Q19 state of these sizes is stored with the streaming (non-temporal) policy: it is
// when one state buffer exceeds the Infinity Cache, where it measured 4.5% faster at 256^3 FP32.
template <typename T, int NC>
inline bool stream_stores3d(const StepArgs<T>& a)
{
    return (int64_t)a.nz * plane3d_elems(a.nx, a.ny, 19 * NC) * (int64_t)sizeof(T) > kStreamStoreBytes;
}

// Launch of the NC-component kernels (one translation unit per set of NC).
template <typename T, int NC>
hipError_t launch_step3d_n(const StepArgs<T>& a, int width, int height, int variant, bool mrt, hipStream_t s)
{
    dim3 grid(a.nitems);
    const bool nt = stream_stores3d<T, NC>(a);
#define TLB_L3(BX, BY, V, M)                                                                         \
    if (width == BX && height == BY && variant == V && mrt == M) {                                   \
        if (nt)                                                                                      \
            hipLaunchKernelGGL((k_step3d<T, BX, BY, V, M, NC, true>), grid, dim3(BX * BY), 0, s, a); \
        else                                                                                         \
            hipLaunchKernelGGL((k_step3d<T, BX, BY, V, M, NC, false>), grid, dim3(BX * BY), 0, s, a);\
        return hipGetLastError();                                                                    \
    }
    TLB_L3(32, 8, 0, false)
    TLB_L3(64, 4, 0, false)
    TLB_L3(32, 8, 1, false)
    TLB_L3(64, 4, 1, false)
    TLB_L3(32, 8, 0, true)
    TLB_L3(64, 4, 0, true)
    TLB_L3(32, 8, 1, true)
    TLB_L3(64, 4, 1, true)
    if constexpr (sizeof(T) == 4 && NC <= 4) {  // VAR 2: FP32 storage of three or four components
        TLB_L3(32, 8, 2, false)
        TLB_L3(64, 4, 2, false)
        TLB_L3(32, 8, 2, true)
        TLB_L3(64, 4, 2, true)
    }
#undef TLB_L3
    return hipErrorInvalidValue;
}

}  // namespace tlb
