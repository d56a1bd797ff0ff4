// Strip sweep of the fused D2Q9 ternary LB step for gfx950: pull propagation + half-way
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
// Every other step (A.flip) reverses all directions, so that a chunk first
// reads the rows it wrote last in the previous step, which are the likeliest
// to be still in the Infinity Cache.
// The concentration deviations dC_m of the last four rows of the sweep sit in
// LDS (W+2 entries per row: the strip and one halo column on each side).  Per
// row the lane needs S = C(x-1) + C(x+1) and D = C(x+1) - C(x-1), which fold
// the 9-point stencils into
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
#pragma once

#include "tlb_internal.hpp"

namespace tlb {

using L9 = D2Q9;

// Addressing of population array j (= 9 s + i) of a species-major state [NC][9][N].  A state of at
// most 4 GiB is covered by one buffer descriptor and a wavefront-uniform byte offset
// (j N + row) sizeof(T).  A larger state (BIG) takes one descriptor per array, so that byte offsets
// within an array (row y * nx + column) stay below 2^32 whatever the size of the whole state; the
// extra scalar work of building them costs about 2% at 1024^2, hence the two forms.
template <typename T, bool BIG>
struct StateAddr {
    const T* base;
    int64_t N;
    Rsrc whole;
    __device__ __forceinline__ StateAddr(const T* b, int64_t n, int nc) : base(b), N(n)
    {
        whole = make_rsrc(b, BIG ? 0u : (uint32_t)((int64_t)9 * nc * n * (int64_t)sizeof(T)));
    }
    __device__ __forceinline__ Rsrc rsrc(int j) const
    {
        return BIG ? make_rsrc(base + (int64_t)j * N, (uint32_t)(N * (int64_t)sizeof(T))) : whole;
    }
    // byte offset of row element `row` (= y nx) of array j
    __device__ __forceinline__ uint32_t soff(int j, uint32_t row) const
    {
        return (uint32_t)((BIG ? row : (uint32_t)j * (uint32_t)N + row) * (uint32_t)sizeof(T));
    }
};

// Pull of the post-propagation populations of row y at the lane's column:
// f_i(r) = u_i(r - e_i), or u_opp(i)(r) when r - e_i lies beyond a wall
// (half-way bounce-back).  vo[0..2]: byte offsets of columns x, x-1, x+1;
// every row-dependent part of the address is wavefront-uniform.
template <typename T, int NC = 3, bool BIG = false>
__device__ __forceinline__ void pull2d(const StepArgs<T>& A, const StateAddr<T, BIG>& src, const uint32_t* vo, int y,
                                       T* p)
{
    const int ny = A.ny;
    const uint32_t nx = (uint32_t)A.nx;
    const uint32_t ym = (y == 0) ? ny - 1 : y - 1;
    const uint32_t yp = (y == ny - 1) ? 0 : y + 1;
    const bool blo = A.walls && y == 0;
    const bool bhi = A.walls && y == ny - 1;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int ex = L9::ex[i], ey = L9::ey[i];
        const bool bb = (ey == 1) ? blo : (ey == -1) ? bhi : false;
        const uint32_t ys = ey == 0 ? (uint32_t)y : (ey == 1 ? ym : yp);
        const int ia = bb ? L9::opp[i] : i;
        const uint32_t row = bb ? (uint32_t)y * nx : ys * nx;
        const uint32_t v = bb ? vo[0] : vo[ex == 0 ? 0 : (ex == 1 ? 1 : 2)];
#pragma unroll
        for (int s = 0; s < NC; ++s)
            p[9 * s + i] = bload<T>(src.rsrc(9 * s + ia), v, src.soff(9 * s + ia, row));
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

// The D2Q9 stencils of one node from three rows of C: a and c are the rows
// before and after the node's row b in sweep order (dir > 0: a is row y-1),
// each given as the node's column c, S = left + right and D = right - left.
// Every sum is symmetric in a and c except the y differences, which take the
// rows' true order, so both sweep directions round identically.
template <typename C>
__device__ __forceinline__ void stencil9(C ac, C aS, C aD, C bc, C bS, C bD, C cc, C cS, C cD, int dir, C* g, C& lap)
{
    const C up = dir > 0 ? cc : ac, dn = dir > 0 ? ac : cc;
    const C Sup = dir > 0 ? cS : aS, Sdn = dir > 0 ? aS : cS;
    g[0] = bD * C(1.0 / 3.0) + (aD + cD) * C(1.0 / 12.0);
    g[1] = (up - dn) * C(1.0 / 3.0) + (Sup - Sdn) * C(1.0 / 12.0);
    g[2] = C(0);
    lap = (bS + (ac + cc)) * C(2.0 / 3.0) + (aS + cS) * C(1.0 / 6.0) - bc * C(10.0 / 3.0);
}

// Occupancy target (wavefronts per SIMD) the register allocation is held to
// (the arithmetic is FP64 for both storage types).
template <typename T, int DEPTH>
constexpr int step2d_waves(int nc = 3) { return (DEPTH || nc > 3) ? 1 : 2; }

template <typename T, int W, int NC = 3>
struct Sweep2Lds {
    // Rows of dC_m (arithmetic precision) in sweep order, four rotating
    // buffers; slot 0 and slot nact+1 hold the halo columns, slot t+1 lane
    // t's own column.
    acc_t<T> row[4][NC][W + 2];
    T hsc[2][2][9 * NC];  // halo populations [buf][left/right][j]
};

// One work item: strip `strip` (W columns) of rows [chunk*A.chunk, ...) of
// the lattice described by A, swept in the direction given by the chunk's
// parity.  Every lane of the workgroup must call it.
template <typename T, int W, int DEPTH, bool MRT = false, int NC = 3, bool BIG = false>
__device__ __forceinline__ void sweep2d(const StepArgs<T>& A, int strip, int chunk, Sweep2Lds<T, W, NC>& S)
{
    auto& lds = S.row;
    auto& hsc = S.hsc;
    const int t = threadIdx.x;
    const int x0 = strip * W;
    const int nact = min(W, A.nx - x0);
    const bool active = t < nact;
    const int x = x0 + (active ? t : nact - 1);
    const int y0 = chunk * A.chunk;
    const int y1 = min(y0 + A.chunk, A.ny);
    const int L = y1 - y0;
    const int dir = ((chunk ^ A.flip) & 1) ? -1 : 1;
    const int yfirst = dir > 0 ? y0 : y1 - 1;
    const bool hl = (t == 0);
    const bool hr = (t == nact - 1);
    const int xl = (x0 == 0) ? A.nx - 1 : x0 - 1;
    const int xr = (x0 + nact == A.nx) ? 0 : x0 + nact;
    // cooperative halo loaders: the J = 9 NC populations of the left halo node
    // are pulled by lanes 0 .. J-1 of the first wavefront, those of the right
    // one by lanes 32 .. 32+J-1 of the last when J <= 32 (distinct lanes, one
    // held value per lane), else by lanes 64-J .. 63 (with one wavefront a lane
    // may then load for both sides and holds two values)
    constexpr int J = 9 * NC;
    constexpr bool one_held = J <= 32;
    constexpr int HR = one_held ? 0 : 1;  // slot of the right-side value
    const int lane = t & 63;
    const bool ldl = (t < 64) && lane < J;
    const bool ldr = one_held ? ((t >= W - 64) && lane >= 32 && lane < 32 + J) : ((t >= W - 64) && lane >= 64 - J);
    const int hjl = lane, hjr = one_held ? lane - 32 : lane - (64 - J);
    const uint32_t nxz = (uint32_t)A.nx;  // nz == 1

    const StateAddr<T, BIG> src(A.src, A.N, NC), dst(A.dst, A.N, NC);

    // Row r_j of the sweep (j = -1 .. L) lives in LDS buffer (j + 1) & 3.
    auto row_of = [&](int j) { return yfirst + j * dir; };
    auto ghost_of = [&](int y) { return (A.walls && y < 0) ? 0 : ((A.walls && y >= A.ny) ? 1 : -1); };
    auto wrap_y = [&](int y) { return y < 0 ? y + A.ny : (y >= A.ny ? y - A.ny : y); };

    const uint32_t vo[3] = {(uint32_t)x * (uint32_t)sizeof(T),
                            (uint32_t)(x == 0 ? A.nx - 1 : x - 1) * (uint32_t)sizeof(T),
                            (uint32_t)(x == A.nx - 1 ? 0 : x + 1) * (uint32_t)sizeof(T)};

    // Three population buffers that take turns as: the row being collided,
    // the next row, and (DEPTH = 1) the row being prefetched.  The sweep loop
    // is unrolled so that the roles rotate without register copies.
    using C = acc_t<T>;
    T P0[J], P1[J], P2[J];
#pragma unroll
    for (int i = 0; i < J; ++i) P0[i] = P1[i] = P2[i] = T(0);
    Moments<C, NC> M0, M1, M2;
    // halo populations held by a loader lane per buffer (left, and right in slot HR)
    T Hb0[HR + 1], Hb1[HR + 1], Hb2[HR + 1];
#pragma unroll
    for (int q = 0; q <= HR; ++q) Hb0[q] = Hb1[q] = Hb2[q] = T(0);
    int hb = 0;

    auto load_row = [&](int y, T* p, T* hv) {
        if (active) pull2d<T, NC, BIG>(A, src, vo, y, p);
        if constexpr (one_held) {
            if (ldl || ldr) hv[0] = pull2d_one<T>(A, ldl ? hjl : hjr, ldl ? xl : xr, y);
        } else {
            if (ldl) hv[0] = pull2d_one<T>(A, hjl, xl, y);
            if (ldr) hv[HR] = pull2d_one<T>(A, hjr, xr, y);
        }
    };

    // Fluid row into buffer q: own dC and the halo populations to LDS, a
    // barrier, then the lanes next to the halo sum the gathered populations
    // (in the same order as every node) into the halo slots.
    auto finish_fluid = [&](const T* p, const T* hv, int q, Moments<C, NC>& mo) {
        mo = moments<L9, NC>(p, p + 9, p + 18);
        C c[NC];
        conc_dev<C, NC>(mo, c);
        if (active) {
#pragma unroll
            for (int m = 0; m < NC; ++m) lds[q][m][t + 1] = c[m];
        }
        if constexpr (one_held) {
            if (ldl || ldr) hsc[hb][ldl ? 0 : 1][ldl ? hjl : hjr] = hv[0];
        } else {
            if (ldl) hsc[hb][0][hjl] = hv[0];
            if (ldr) hsc[hb][1][hjr] = hv[HR];
        }
        __syncthreads();
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            if ((side == 0 && hl) || (side == 1 && hr)) {
                T v[J];
#pragma unroll
                for (int j = 0; j < J; ++j) v[j] = hsc[hb][side][j];
                const Moments<C, NC> hm = moments<L9, NC>(v, v + 9, v + 18);
                C hc[NC];
                conc_dev<C, NC>(hm, hc);
                const int slot = side == 0 ? 0 : nact + 1;
#pragma unroll
                for (int m = 0; m < NC; ++m) lds[q][m][slot] = hc[m];
            }
        }
        hb ^= 1;
    };
    // Ghost row beyond wall w into buffer q from the adjacent fluid row in
    // buffer qa (reading R8): C_m(ghost) = C_m(adjacent) + h_m / (alpha^2 kappa_m).
    auto finish_ghost = [&](int w, int qa, int q) {
        const T* __restrict__ wt = A.wet + (size_t)w * NC * nxz;
        if (active) {
#pragma unroll
            for (int m = 0; m < NC; ++m) lds[q][m][t + 1] = lds[qa][m][t + 1] + C(wt[m * nxz + x]);
        }
#pragma unroll
        for (int m = 0; m < NC; ++m) {
            if (hl) lds[q][m][0] = lds[qa][m][0] + C(wt[m * nxz + xl]);
            if (hr) lds[q][m][nact + 1] = lds[qa][m][nact + 1] + C(wt[m * nxz + xr]);
        }
        __syncthreads();
    };

    // One row of the sweep: Pc/Mc hold row r_j, Pn row r_{j+1} (in flight),
    // Pp receives row r_{j+2} (DEPTH = 1).
    auto row_step = [&](int j, T* Pc, Moments<C, NC>& Mc, T* Pn, Moments<C, NC>& Mn, T* Hn, T* Pp, T* Hp) {
        const int y = row_of(j);
        const int qa = j & 3, qb = (j + 1) & 3, qc = (j + 2) & 3;
        const int yc = row_of(j + 1);
        const int gc = ghost_of(yc);
        if constexpr (DEPTH == 0) {
            if (gc < 0 && j > 0) load_row(wrap_y(yc), Pn, Hn);
        }
        if (gc < 0)
            finish_fluid(Pn, Hn, qc, Mn);
        else
            finish_ghost(gc, qb, qc);
        if constexpr (DEPTH == 1) {
            const int yn = row_of(j + 2);
            if (j + 2 <= L && ghost_of(yn) < 0) load_row(wrap_y(yn), Pp, Hp);
        }
        if (active) {
            // Stencils of row y from the three rows in LDS (qa: previous row in
            // sweep order, qc: next one).
            C gC[NC][3], lC[NC];
#pragma unroll
            for (int m = 0; m < NC; ++m) {
                const C ac = lds[qa][m][t + 1], aS = lds[qa][m][t] + lds[qa][m][t + 2],
                        aD = lds[qa][m][t + 2] - lds[qa][m][t];
                const C bc = lds[qb][m][t + 1], bS = lds[qb][m][t] + lds[qb][m][t + 2],
                        bD = lds[qb][m][t + 2] - lds[qb][m][t];
                const C cc = lds[qc][m][t + 1], cS = lds[qc][m][t] + lds[qc][m][t + 2],
                        cD = lds[qc][m][t + 2] - lds[qc][m][t];
                stencil9<C>(ac, aS, aD, bc, bS, bD, cc, cS, cD, dir, gC[m], lC[m]);
            }
            C dc[NC];
#pragma unroll
            for (int m = 0; m < NC; ++m) dc[m] = lds[qb][m][t + 1];
            collide<L9, MRT, NC>(A.P, Mc, dc, gC, lC, Pc, Pc + 9, Pc + 18);
            const uint32_t row = (uint32_t)y * (uint32_t)A.nx;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
#pragma unroll
                for (int s = 0; s < NC; ++s)
                    bstore<T>(Pc[9 * s + i], dst.rsrc(9 * s + i), vo[0], dst.soff(9 * s + i, row));
            }
        }
    };

    // Prologue: rows r_{-1} (LDS buffer 0) and r_0 (buffer 1, populations in
    // P0); the pull of r_1 into P1.
    {
        const int ya = row_of(-1);
        const int ga = ghost_of(ya);
        if (ga < 0) {
            load_row(wrap_y(ya), P1, Hb1);
            finish_fluid(P1, Hb1, 0, M1);
            load_row(yfirst, P0, Hb0);
            finish_fluid(P0, Hb0, 1, M0);
        } else {
            load_row(yfirst, P0, Hb0);
            finish_fluid(P0, Hb0, 1, M0);
            finish_ghost(ga, 1, 0);
        }
        const int yc = row_of(1);
        if (ghost_of(yc) < 0) load_row(wrap_y(yc), P1, Hb1);
    }

    if constexpr (DEPTH == 0) {
        int j = 0;
        for (; j + 1 < L; j += 2) {
            row_step(j, P0, M0, P1, M1, Hb1, P2, Hb2);
            row_step(j + 1, P1, M1, P0, M0, Hb0, P2, Hb2);
        }
        if (j < L) row_step(j, P0, M0, P1, M1, Hb1, P2, Hb2);
    } else {
        int j = 0;
        for (; j + 2 < L; j += 3) {
            row_step(j, P0, M0, P1, M1, Hb1, P2, Hb2);
            row_step(j + 1, P1, M1, P2, M2, Hb2, P0, Hb0);
            row_step(j + 2, P2, M2, P0, M0, Hb0, P1, Hb1);
        }
        if (j < L) row_step(j, P0, M0, P1, M1, Hb1, P2, Hb2);
        if (j + 1 < L) row_step(j + 1, P1, M1, P2, M2, Hb2, P0, Hb0);
    }
}

}  // namespace tlb
