// Fused D2Q9 ternary LB step for gfx950: pull propagation + half-way
// bounce-back, moments, wetting ghost rows, lattice stencils, local
// thermodynamics, equilibria and BGK collision in one pass over HBM.
//
// State: u_t = post-collision populations of the previous step, SoA
// [species][q][n] (shifted storage, see tlb_device.hpp).  One launch maps
// u_t -> u_{t+1}; the post-propagation state s_t is the pull of u_t.
//
// Work decomposition.  A workgroup of W lanes (W = 64, 128 or 256) owns a
// strip of W columns and sweeps `chunk` rows upwards.  Lane t keeps its own
// column's concentration deviations dC_m for rows y-1, y, y+1 in registers;
// the x-neighbours come from a double-buffered LDS row of W+2 entries (one
// halo column on each side, computed by lanes 0 and W-1 in an extra pull).
// Per row the lane needs from LDS only S = C(x-1) + C(x+1) and
// D = C(x+1) - C(x-1), which fold the 9-point stencils into
//   d_x C   = D_y/3 + (D_{y-1} + D_{y+1})/12
//   d_y C   = (C_{y+1} - C_{y-1})/3 + (S_{y+1} - S_{y-1})/12
//   lap C   = 2/3 (S_y + C_{y-1} + C_{y+1}) + (S_{y-1} + S_{y+1})/6 - 10/3 C_y
// (the isotropic stencils d_a X = 3 sum w_i e_ia X(r+e_i),
//  lap X = 6 sum w_i [X(r+e_i) - X(r)] written out for D2Q9).
// HBM traffic per node and step: 27 values read (pull) + 27 written; the
// halo rows at chunk ends and the two halo columns are re-read from L2.
#include "tlb_internal.hpp"

namespace tlb {

using L9 = D2Q9;

// Pull the post-propagation populations of node (x, y): f_i(r) = u_i(r - e_i),
// or u_opp(i)(r) when r - e_i lies beyond a wall (half-way bounce-back).
template <typename T>
__device__ __forceinline__ void pull2d(const StepArgs<T>& A, int x, int y, T* f, T* g, T* k)
{
    const int nx = A.nx, ny = A.ny;
    const int xm = (x == 0) ? nx - 1 : x - 1;
    const int xp = (x == nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? ny - 1 : y - 1;
    const int yp = (y == ny - 1) ? 0 : y + 1;
    const bool blo = A.walls && y == 0;
    const bool bhi = A.walls && y == ny - 1;
    const uint32_t N = (uint32_t)A.N;
    const uint32_t n0 = (uint32_t)y * nx + x;
    const T* __restrict__ src = A.src;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const T* __restrict__ b = src + (int64_t)s * 9 * A.N;
        T* out = (s == 0) ? f : (s == 1) ? g : k;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int ex = L9::ex[i], ey = L9::ey[i];
            const bool bb = (ey == 1) ? blo : (ey == -1) ? bhi : false;
            const int xs = ex == 0 ? x : (ex == 1 ? xm : xp);
            const int ys = ey == 0 ? y : (ey == 1 ? ym : yp);
            const uint32_t off = bb ? (uint32_t)L9::opp[i] * N + n0 : (uint32_t)i * N + (uint32_t)ys * nx + xs;
            out[i] = b[off];
        }
    }
}

template <typename T>
struct Row2 {
    T c[3];  // own dC_m
    T S[3];  // dC(x-1) + dC(x+1)
    T D[3];  // dC(x+1) - dC(x-1)
};

// HOLD = true keeps the pulled populations of row y+1 in registers until the
// row is collided one iteration later; HOLD = false keeps only the moments
// and pulls the row again (from cache) when it is collided, which halves the
// live state and raises occupancy.
template <typename T, int W, bool HOLD>
__global__ __launch_bounds__(W) void k_step2d(StepArgs<T> A)
{
    __shared__ T lds[2][3][W + 2];

    const int item = xcd_item(blockIdx.x, A.nitems);
    const int strip = item / A.nchunks;
    const int chunk = item - strip * A.nchunks;
    const int t = threadIdx.x;
    const int x0 = strip * W;
    const int nact = min(W, A.nx - x0);
    const bool active = t < nact;
    const int x = x0 + (active ? t : nact - 1);
    const int y0 = chunk * A.chunk;
    const int y1 = min(y0 + A.chunk, A.ny);
    const bool hl = (t == 0);
    const bool hr = (t == nact - 1);
    const int xl = (x0 == 0) ? A.nx - 1 : x0 - 1;
    const int xr = (x0 + nact == A.nx) ? 0 : x0 + nact;
    const uint32_t nxz = (uint32_t)A.nx;  // nz == 1

    T fb[9], gb[9], kb[9];  // HOLD: populations of row y
    T fc[9], gc[9], kc[9];  // pull buffer (row y + 1)
    Row2<T> ra, rb, rc;
    T hcl[3], hcr[3];  // halo-column dC of the most recent row (for ghost rows)
    int buf = 0;

    // Publish a row: own dC to LDS slot t+1, halo dC to slots 0 / nact+1;
    // then read back the neighbour sums.
    auto publish = [&](Row2<T>& r) {
        if (active) {
#pragma unroll
            for (int m = 0; m < 3; ++m) lds[buf][m][t + 1] = r.c[m];
        }
        if (hl) {
#pragma unroll
            for (int m = 0; m < 3; ++m) lds[buf][m][0] = hcl[m];
        }
        if (hr) {
#pragma unroll
            for (int m = 0; m < 3; ++m) lds[buf][m][nact + 1] = hcr[m];
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const T l = lds[buf][m][t];
            const T rr = lds[buf][m][t + 2];
            r.S[m] = l + rr;
            r.D[m] = rr - l;
        }
        buf ^= 1;
    };

    // A fluid row: pull own column (populations left in fc/gc/kc) and the halo columns.
    auto fluid_row = [&](int y, Row2<T>& r) {
        pull2d<T>(A, x, y, fc, gc, kc);
        const Moments<T> mo = moments<L9, T>(fc, gc, kc);
        conc_dev<T>(mo, r.c);
        if (hl) {
            T hf[9], hg[9], hk[9];
            pull2d<T>(A, xl, y, hf, hg, hk);
            const Moments<T> hm = moments<L9, T>(hf, hg, hk);
            conc_dev<T>(hm, hcl);
        }
        if (hr) {
            T hf[9], hg[9], hk[9];
            pull2d<T>(A, xr, y, hf, hg, hk);
            const Moments<T> hm = moments<L9, T>(hf, hg, hk);
            conc_dev<T>(hm, hcr);
        }
        publish(r);
    };

    auto hold = [&]() {
        if constexpr (HOLD) {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                fb[i] = fc[i];
                gb[i] = gc[i];
                kb[i] = kc[i];
            }
        }
    };

    // A ghost row beyond wall w, from the adjacent fluid row (reading R8):
    // C_m(ghost) = C_m(adjacent) + h_m / (alpha^2 kappa_m).
    auto ghost_row = [&](int w, const Row2<T>& adj, Row2<T>& r) {
        const T* __restrict__ wt = A.wet + (size_t)w * 3 * nxz;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            r.c[m] = adj.c[m] + wt[m * nxz + x];
            if (hl) hcl[m] += wt[m * nxz + xl];
            if (hr) hcr[m] += wt[m * nxz + xr];
        }
        publish(r);
    };

    // Prologue: rows y0 - 1 and y0.
    if (A.walls && y0 == 0) {
        fluid_row(0, rb);
        hold();
        ghost_row(0, rb, ra);
    } else {
        const int ya = (y0 == 0) ? A.ny - 1 : y0 - 1;
        fluid_row(ya, ra);
        fluid_row(y0, rb);
        hold();
    }

    const uint32_t N = (uint32_t)A.N;
    for (int y = y0; y < y1; ++y) {
        // Row y + 1: a fluid row, or the ghost row above the top wall.
        if (A.walls && y + 1 == A.ny) {
            ghost_row(1, rb, rc);
        } else {
            const int yn = (y + 1 == A.ny) ? 0 : y + 1;
            fluid_row(yn, rc);
        }

        // Stencils of row y.
        T gC[3][3], lC[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            gC[m][0] = rb.D[m] * T(1.0 / 3.0) + (ra.D[m] + rc.D[m]) * T(1.0 / 12.0);
            gC[m][1] = (rc.c[m] - ra.c[m]) * T(1.0 / 3.0) + (rc.S[m] - ra.S[m]) * T(1.0 / 12.0);
            gC[m][2] = T(0);
            lC[m] = (rb.S[m] + ra.c[m] + rc.c[m]) * T(2.0 / 3.0) + (ra.S[m] + rc.S[m]) * T(1.0 / 6.0) -
                    rb.c[m] * T(10.0 / 3.0);
        }
        if constexpr (!HOLD) pull2d<T>(A, x, y, fb, gb, kb);
        const Moments<T> mb = moments<L9, T>(fb, gb, kb);
        collide<L9, T>(A.P, mb, rb.c, gC, lC, fb, gb, kb);

        if (active) {
            T* __restrict__ dst = A.dst;
            const uint32_t n0 = (uint32_t)y * A.nx + x;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                dst[(uint32_t)i * N + n0] = fb[i];
                dst[(int64_t)9 * A.N + (uint32_t)i * N + n0] = gb[i];
                dst[(int64_t)18 * A.N + (uint32_t)i * N + n0] = kb[i];
            }
        }

        ra = rb;
        rb = rc;
        hold();
    }
}

template <typename T>
hipError_t launch_step2d(const StepArgs<T>& a, int width, int hold, hipStream_t s)
{
    dim3 grid(a.nitems);
#define TLB_L2(W, H)                                                               \
    if (width == W && (hold != 0) == H) {                                          \
        hipLaunchKernelGGL((k_step2d<T, W, H>), grid, dim3(W), 0, s, a);           \
        return hipGetLastError();                                                  \
    }
    TLB_L2(64, false)
    TLB_L2(128, false)
    TLB_L2(256, false)
    TLB_L2(64, true)
    TLB_L2(128, true)
    TLB_L2(256, true)
#undef TLB_L2
    return hipErrorInvalidValue;
}

template hipError_t launch_step2d<float>(const StepArgs<float>&, int, int, hipStream_t);
template hipError_t launch_step2d<double>(const StepArgs<double>&, int, int, hipStream_t);

}  // namespace tlb
