// Fused D2Q9 ternary LB step for gfx950: pull propagation + half-way
// bounce-back, moments, wetting ghost rows, lattice stencils, local
// thermodynamics, equilibria and BGK collision in one pass over HBM.
//
// State: u_t = post-collision populations of the previous step, SoA
// [species][q][n] (shifted storage, see tlb_device.hpp).  One launch maps
// u_t -> u_{t+1}; the post-propagation state s_t is the pull of u_t.
//
// Work decomposition.  A workgroup of W lanes (W = 64, 128 or 256) owns a
// strip of W columns and sweeps a chunk of rows, upwards for even chunks and
// downwards for odd ones, so that two neighbouring chunks reach their shared
// boundary rows at the same time and the second read of those rows hits L2.
// Lane t keeps its own column's concentration deviations dC_m for three
// consecutive rows in registers; the x-neighbours come from a double-buffered
// LDS row.  Per row the lane needs from LDS only S = C(x-1) + C(x+1) and
// D = C(x+1) - C(x-1), which fold the 9-point stencils into
//   d_x C = D_y/3 + (D_{y-1} + D_{y+1})/12
//   d_y C = (C_{y+1} - C_{y-1})/3 + (S_{y+1} - S_{y-1})/12
//   lap C = 2/3 (S_y + (C_{y-1} + C_{y+1})) + (S_{y-1} + S_{y+1})/6 - 10/3 C_y
// (the isotropic stencils d_a X = 3 sum w_i e_ia X(r+e_i),
//  lap X = 6 sum w_i [X(r+e_i) - X(r)] written out for D2Q9), grouped so that
// both sweep directions round identically.
//
// The columns x0-1 and x0+W of the neighbouring strips are gathered
// cooperatively: lanes 0..26 of the first wavefront load the 27 populations
// of the left halo node (one each) and lanes 32..58 of the last wavefront
// those of the right one; the values pass through LDS to the lane next to
// the halo, which sums them in the same order as every other node.
//
// DEPTH = 1 software-pipelines the sweep: the pull of row r+2 is issued
// before row r is collided, so the HBM reads overlap the arithmetic.
// HBM traffic per node and step: 27 values read (pull) + 27 written.
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
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const T* __restrict__ b = A.src + (int64_t)s * 9 * A.N;
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

// One population (species s = j / 9, direction i = j % 9) of the pull of node (x, y).
template <typename T>
__device__ __forceinline__ T pull2d_one(const StepArgs<T>& A, int j, int x, int y)
{
    // e_x + 1, e_y + 1 and opp(i) of the D2Q9 order, packed 2 / 2 / 4 bits per direction
    constexpr uint32_t EXP = 1u | 2u << 2 | 0u << 4 | 1u << 6 | 1u << 8 | 2u << 10 | 2u << 12 | 0u << 14 | 0u << 16;
    constexpr uint32_t EYP = 1u | 1u << 2 | 1u << 4 | 2u << 6 | 0u << 8 | 2u << 10 | 0u << 12 | 2u << 14 | 0u << 16;
    constexpr uint64_t OPP = 0ull | 2ull << 4 | 1ull << 8 | 4ull << 12 | 3ull << 16 | 8ull << 20 | 7ull << 24 |
                             6ull << 28 | 5ull << 32;
    const int s = j / 9, i = j - 9 * s;
    const int ex = (int)((EXP >> (2 * i)) & 3u) - 1;
    const int ey = (int)((EYP >> (2 * i)) & 3u) - 1;
    const int op = (int)((OPP >> (4 * i)) & 15u);
    const int nx = A.nx, ny = A.ny;
    int xs = x - ex;
    xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
    int ys = y - ey;
    int64_t off;
    if (A.walls && (ys < 0 || ys >= ny)) {
        off = (int64_t)op * A.N + (int64_t)y * nx + x;
    } else {
        ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
        off = (int64_t)i * A.N + (int64_t)ys * nx + xs;
    }
    return A.src[(int64_t)s * 9 * A.N + off];
}

template <typename T>
struct Row2 {
    T c[3];  // own dC_m
    T S[3];  // dC(x-1) + dC(x+1)
    T D[3];  // dC(x+1) - dC(x-1)
};

template <typename T, int W, int DEPTH>
__global__ __launch_bounds__(W) void k_step2d(StepArgs<T> A)
{
    __shared__ T lds[2][3][W];
    __shared__ T hsc[2][2][27];  // halo populations [buf][left/right][j]

    const int item = xcd_item(blockIdx.x, A.nitems);
    const int chunk = item / A.ntx;  // chunk-major: an XCD's range covers whole bands
    const int strip = item - chunk * A.ntx;
    const int t = threadIdx.x;
    const int x0 = strip * W;
    const int nact = min(W, A.nx - x0);
    const bool active = t < nact;
    const int x = x0 + (active ? t : nact - 1);
    const int y0 = chunk * A.chunk;
    const int y1 = min(y0 + A.chunk, A.ny);
    const int L = y1 - y0;
    const int dir = (chunk & 1) ? -1 : 1;
    const int yfirst = dir > 0 ? y0 : y1 - 1;
    const bool hl = (t == 0);
    const bool hr = (t == nact - 1);
    const int xl = (x0 == 0) ? A.nx - 1 : x0 - 1;
    const int xr = (x0 + nact == A.nx) ? 0 : x0 + nact;
    // cooperative halo loaders
    const int lane = t & 63;
    const bool ldl = (t < 64) && lane < 27;
    const bool ldr = (t >= W - 64) && lane >= 32 && lane < 59;
    const int hj = ldl ? lane : lane - 32;
    const int hx = ldl ? xl : xr;
    const int hside = ldl ? 0 : 1;
    const uint32_t nxz = (uint32_t)A.nx;  // nz == 1
    const uint32_t N = (uint32_t)A.N;

    // Row r_j of the sweep (j = -1 .. L); kind: -1 fluid, 0/1 ghost of that wall.
    auto row_of = [&](int j) { return yfirst + j * dir; };
    auto ghost_of = [&](int y) { return (A.walls && y < 0) ? 0 : ((A.walls && y >= A.ny) ? 1 : -1); };
    auto wrap_y = [&](int y) { return y < 0 ? y + A.ny : (y >= A.ny ? y - A.ny : y); };

    T pB[27], pC[27], pN[27];  // populations: row being collided, next row, prefetched row
#pragma unroll
    for (int i = 0; i < 27; ++i) pB[i] = pC[i] = pN[i] = T(0);
    T hvC = T(0), hvN = T(0);  // halo population held by a loader lane (next / prefetched row)
    Row2<T> ra, rb, rc;
    T hcl[3], hcr[3];  // halo dC of the most recent fluid row (lanes 0 / nact-1)
    int buf = 0;

    auto load_row = [&](int y, T* p, T& hv) {
        if (active) pull2d<T>(A, x, y, p, p + 9, p + 18);
        if (ldl || ldr) hv = pull2d_one<T>(A, hj, hx, y);
    };

    // Publish a row: own dC and (for a fluid row) the halo populations to
    // LDS; after the barrier read the neighbour sums.  The lanes next to the
    // halo build the halo dC from the gathered populations.
    auto publish = [&](Row2<T>& r, bool fluid, int gw) {
        if (active) {
#pragma unroll
            for (int m = 0; m < 3; ++m) lds[buf][m][t] = r.c[m];
        }
        if (fluid && (ldl || ldr)) hsc[buf][hside][hj] = hvC;
        __syncthreads();
        if (fluid && (hl || hr)) {
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                if ((side == 0 && hl) || (side == 1 && hr)) {
                    T q[27];
#pragma unroll
                    for (int j = 0; j < 27; ++j) q[j] = hsc[buf][side][j];
                    const Moments<T> hm = moments<L9, T>(q, q + 9, q + 18);
                    conc_dev<T>(hm, side == 0 ? hcl : hcr);
                }
            }
        }
        if (!fluid) {
            const T* __restrict__ wt = A.wet + (size_t)gw * 3 * nxz;
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                if (hl) hcl[m] += wt[m * nxz + xl];
                if (hr) hcr[m] += wt[m * nxz + xr];
            }
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const T l = hl ? hcl[m] : lds[buf][m][t > 0 ? t - 1 : 0];
            const T rr = hr ? hcr[m] : lds[buf][m][t + 1 < W ? t + 1 : W - 1];
            r.S[m] = l + rr;
            r.D[m] = rr - l;
        }
        buf ^= 1;
    };

    // Finish row y whose populations are in p (moments -> dC -> publish).
    auto finish_fluid = [&](const T* p, Row2<T>& r) {
        const Moments<T> mo = moments<L9, T>(p, p + 9, p + 18);
        conc_dev<T>(mo, r.c);
        publish(r, true, 0);
    };
    // Ghost row beyond wall w from the adjacent fluid row (reading R8):
    // C_m(ghost) = C_m(adjacent) + h_m / (alpha^2 kappa_m).
    auto finish_ghost = [&](int w, const Row2<T>& adj, Row2<T>& r) {
        const T* __restrict__ wt = A.wet + (size_t)w * 3 * nxz;
#pragma unroll
        for (int m = 0; m < 3; ++m) r.c[m] = adj.c[m] + wt[m * nxz + x];
        publish(r, false, w);
    };

    // Prologue: rows r_{-1} (ra) and r_0 (rb, populations in pB); prefetch r_1.
    {
        const int ya = row_of(-1);
        const int ga = ghost_of(ya);
        if (ga < 0) {
            load_row(wrap_y(ya), pC, hvC);
            finish_fluid(pC, ra);
            load_row(yfirst, pB, hvC);
            finish_fluid(pB, rb);
        } else {
            load_row(yfirst, pB, hvC);
            finish_fluid(pB, rb);
            finish_ghost(ga, rb, ra);
        }
        const int yc = row_of(1);
        if (ghost_of(yc) < 0) load_row(wrap_y(yc), pC, hvC);
    }

    for (int j = 0; j < L; ++j) {
        const int y = row_of(j);
        // Row r_{j+1}: finish the fluid row already in flight, or build the ghost row.
        const int yc = row_of(j + 1);
        const int gc = ghost_of(yc);
        if constexpr (DEPTH == 0) {
            if (gc < 0 && j > 0) load_row(wrap_y(yc), pC, hvC);
        }
        if (gc < 0)
            finish_fluid(pC, rc);
        else
            finish_ghost(gc, rb, rc);
        // Prefetch row r_{j+2} (needed while j + 2 <= L).
        if constexpr (DEPTH == 1) {
            const int yn = row_of(j + 2);
            if (j + 2 <= L && ghost_of(yn) < 0) load_row(wrap_y(yn), pN, hvN);
        }

        // Stencils of row y (ra: previous row in sweep order, rc: next one).
        T gC[3][3], lC[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const T up = dir > 0 ? rc.c[m] : ra.c[m];
            const T dn = dir > 0 ? ra.c[m] : rc.c[m];
            const T Sup = dir > 0 ? rc.S[m] : ra.S[m];
            const T Sdn = dir > 0 ? ra.S[m] : rc.S[m];
            gC[m][0] = rb.D[m] * T(1.0 / 3.0) + (ra.D[m] + rc.D[m]) * T(1.0 / 12.0);
            gC[m][1] = (up - dn) * T(1.0 / 3.0) + (Sup - Sdn) * T(1.0 / 12.0);
            gC[m][2] = T(0);
            lC[m] = (rb.S[m] + (ra.c[m] + rc.c[m])) * T(2.0 / 3.0) + (ra.S[m] + rc.S[m]) * T(1.0 / 6.0) -
                    rb.c[m] * T(10.0 / 3.0);
        }
        if (active) {
            const Moments<T> mb = moments<L9, T>(pB, pB + 9, pB + 18);
            collide<L9, T>(A.P, mb, rb.c, gC, lC, pB, pB + 9, pB + 18);
            T* __restrict__ dst = A.dst;
            const uint32_t n0 = (uint32_t)y * A.nx + x;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                dst[(uint32_t)i * N + n0] = pB[i];
                dst[(int64_t)9 * A.N + (uint32_t)i * N + n0] = pB[9 + i];
                dst[(int64_t)18 * A.N + (uint32_t)i * N + n0] = pB[18 + i];
            }
        }

        ra = rb;
        rb = rc;
#pragma unroll
        for (int i = 0; i < 27; ++i) pB[i] = pC[i];
        if constexpr (DEPTH == 1) {
#pragma unroll
            for (int i = 0; i < 27; ++i) pC[i] = pN[i];
            hvC = hvN;
        }
    }
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
