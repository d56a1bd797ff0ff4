// Reverse mode of the fused D2Q9 step: lambda_t = (d u_{t+1} / d u_t)^T lambda_{t+1},
// with the gradients of the wetting parameters h_m (per wall node) and of the
// bulk coefficients kappa_m accumulated on the way.
//
// The forward step is  s = P u  (pull propagation with half-way bounce-back,
// a permutation),  u'(r) = s(r) + omega (E(r) - s(r))  per species, where the
// equilibrium E(r) depends on the node's moments and concentrations and on
// the gradients G_m(r) and Laplacians L_m(r) of C_m over the 9-point
// neighbourhood, including the wetting ghost rows
//   C_m(ghost) = C_m(adjacent) + h_m / (alpha^2 kappa_m).
// Its transpose, for one node r, is
//   1. the moments and concentrations of s_t(r) = (P u_t)(r);
//   2. the local transpose of E and of the relaxation at r, given
//      lambda_{t+1}(r): adjoints of the moments and of C_m used locally
//      (Abar), of the gradients (Gbar_m) and of the Laplacians (Lbar_m), and
//      the direct kappa terms;
//   3. the transposed stencils
//        Cbar_m(r) = Abar_C(r) - 6 (1 - w_0) Lbar_m(r)
//                    + sum_i [3 w_i e_i . Gbar_m(r - e_i) + 6 w_i Lbar_m(r - e_i)],
//      the transpose of the ghost rows (hbar_m += Cbar_ghost / (alpha^2 kappa_m),
//      and the kappa term of the ghost value) and the transpose of the moments,
//      which leave sbar_i(r) = (1 - omega) lambda_{t+1,i}(r) + S(r) + e_i . J(r);
//   4. the transpose of P, written as a gather:
//        lambda_{t,i}(r) = sbar_i(r + e_i), or sbar_opp(i)(r) where r + e_i lies
//      beyond a wall.
// The dependency radius is 3 nodes.  k_adj2d runs all four stages in one
// sweep: a workgroup of K row groups of W lanes covers W columns and produces
// the middle W - 6 of them, sweeping a chunk of rows with the stages one row
// apart (stage 1 at row a, stage 2 at a-1, stage 3 at a-2, stage 4 at a-3),
// K rows per iteration.  The per-row quantities that neighbours need (dC_m;
// Gbar, Lbar; S, J; with K > 1 also the moments and local transposes) live in
// (K + 2)-row LDS rings, the rest in registers.  HBM traffic per node and
// step: u_t and lambda_{t+1} read, lambda_t written (81 values); the
// overlapping halo rows and columns are re-read, from L2 when they are still
// there.
//
// The kappa gradient is summed per work item in a fixed order (lanes, then a
// tree) into its own slot kpart[m][item] (added to it over a reverse pass, or
// written by a single step), which the caller reduces in a fixed order, so
// results do not depend on scheduling.
#include <stdint.h>

#include "../../include/tlb.h"
#include "tlb_internal.hpp"

namespace tlb {

namespace {

using L9 = D2Q9;

__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }
__device__ __forceinline__ int modi(int a, int n)
{
    const int r = a % n;
    return r < 0 ? r + n : r;
}

// Local transpose at one node (stage 2).  Inputs: the node's moments, its dC_m,
// gradients gx, gy and Laplacians lC of C_m, and lambda_{t+1} at the node.
// Outputs: lb = (rho, jx, jy, phi, psi adjoints; Cbar_m used locally) [8],
// bG[m][a] (gradient adjoints), bL[m] (Laplacian adjoints), kb[m] (direct kappa terms).
template <typename T, typename S>
__device__ __forceinline__ void adj_local(const Phys<T>& P, const Moments<T>& mo, const T dc[3], const T gx[3],
                                          const T gy[3], const T lC[3], const S* lam, T lb[8], T bG[3][2], T bL[3],
                                          T kb[3])
{
    // T: arithmetic type; S: storage type of lambda
    const T third = T(1.0 / 3.0);
    T c[3];
    T Txx = 0, Tyy = 0, Txy = 0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        c[m] = third + dc[m];
        Txx += P.a2kappa[m] * gx[m] * gx[m];
        Tyy += P.a2kappa[m] * gy[m] * gy[m];
        Txy += P.a2kappa[m] * gx[m] * gy[m];
    }
    (void)Txx, (void)Tyy, (void)Txy;
    const T rho = T(1) + mo.drho, irho = T(1) / rho;
    const T vx = mo.jx * irho, vy = mo.jy * irho, psi = third + mo.dpsi, vv = vx * vx + vy * vy;
    const T phi = mo.phi;

    // adjoint of the relaxation: Ebar = omega lambda'; rest populations from the mass constraints
    T af[9], ag[9], ak[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        af[i] = P.omega[0] * T(lam[i]);
        ag[i] = P.omega[1] * T(lam[9 + i]);
        ak[i] = P.omega[2] * T(lam[18 + i]);
    }
    T b_drho = af[0], b_phi = ag[0], b_dpsi = ak[0];
    T bA = 0, b_rho = 0, bBp = 0, bBk = 0, b_psi = 0, bTxx = 0, bTyy = 0, bTxy = 0, bvx = 0, bvy = 0, bvv = 0;
    // Opposite directions i and j = opp(i) share the weights w, w^{ab} and the even part
    // Ue = 4.5 (e.v)^2 - 1.5 v^2 of U_i = Ue + Uo, U_j = Ue - Uo (Uo = 3 e_i.v), so each pair enters
    // through the sums and differences of its two adjoints.
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const int j = L9::opp[i];
        if (j < i) continue;
        const T w = T(weight<L9>(i));
        const T fbi = af[i] - af[0], gbi = ag[i] - ag[0], kbi = ak[i] - ak[0];
        const T fbj = af[j] - af[0], gbj = ag[j] - ag[0], kbj = ak[j] - ak[0];
        const T fs = fbi + fbj, fd = fbi - fbj, gs = gbi + gbj, gd = gbi - gbj, ks = kbi + kbj, kd = kbi - kbj;
        const T ev = T(L9::ex[i]) * vx + T(L9::ey[i]) * vy;
        const T Ue = T(4.5) * ev * ev - T(1.5) * vv, Uo = T(3) * ev;
        const T wa = w * P.adv;  // velocity terms of g^eq, k^eq (absent without advection)
        bA += w * fs;
        b_rho += w * (Ue * fs + Uo * fd);
        bTxx += T(3 * wdiag<L9>(i, 0)) * fs;
        bTyy += T(3 * wdiag<L9>(i, 1)) * fs;
        bTxy += T(3 * woff<L9>(i, 0, 1)) * fs;
        bBp += w * gs;
        b_phi += wa * (Ue * gs + Uo * gd);
        bBk += w * ks;
        b_psi += wa * (Ue * ks + Uo * kd);
        // bU = w (rho fb + adv (phi gb + psi kb)) per direction; its pair sum and difference
        const T bUs = w * (rho * fs + P.adv * (phi * gs + psi * ks));
        const T bUd = w * (rho * fd + P.adv * (phi * gd + psi * kd));
        // e_i bU_i (3 + 9 e_i.v) + e_j bU_j (3 + 9 e_j.v) = e_i (3 bUd + 9 (e_i.v) bUs)
        const T bo = T(3) * bUd + T(9) * ev * bUs;
        bvv += T(-1.5) * bUs;
        bvx += T(L9::ex[i]) * bo;
        bvy += T(L9::ey[i]) * bo;
    }
    bvx += T(2) * vx * bvv;
    bvy += T(2) * vy * bvv;
    const T b_jx = bvx * irho, b_jy = bvy * irho;
    b_rho -= (bvx * vx + bvy * vy) * irho;
    b_drho += b_rho;
    b_dpsi += b_psi;
    const T b_pbx = T(3) * bA, b_lam = T(-3) * bA;
    const T bmu_phi = P.gphi3 * bBp, bmu_psi = P.gpsi3 * bBk;
    const T bmu[3] = {T(0.5) * bmu_phi - T(0.5) * bmu_psi, T(-0.5) * bmu_phi - T(0.5) * bmu_psi, bmu_psi};
    b_drho += b_pbx * third;
    const T a2 = P.a2kappa[0] / P.kappa[0];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const T cm = c[m];
        const T q = cm * (T(1) - cm) * (T(1) - T(2) * cm);
        const T dq = T(1) - T(6) * cm + T(6) * cm * cm;
        const T pp = cm * cm * (T(1) - cm) * (T(1) - T(3) * cm);
        const T dp = T(2) * cm - T(12) * cm * cm + T(12) * cm * cm * cm;
        lb[5 + m] = bmu[m] * P.kappa[m] * dq + b_pbx * T(0.5) * P.kappa[m] * dp + b_lam * P.a2kappa[m] * lC[m];
        bL[m] = -P.a2kappa[m] * bmu[m] + b_lam * P.a2kappa[m] * cm;
        bG[m][0] = bTxx * T(2) * P.a2kappa[m] * gx[m] + bTxy * P.a2kappa[m] * gy[m];
        bG[m][1] = bTyy * T(2) * P.a2kappa[m] * gy[m] + bTxy * P.a2kappa[m] * gx[m];
        kb[m] = bmu[m] * (q - a2 * lC[m]) + b_pbx * T(0.5) * pp + b_lam * a2 * cm * lC[m] +
                a2 * (bTxx * gx[m] * gx[m] + bTyy * gy[m] * gy[m] + bTxy * gx[m] * gy[m]);
    }
    lb[0] = b_drho;
    lb[1] = b_jx;
    lb[2] = b_jy;
    lb[3] = b_phi;
    lb[4] = b_dpsi;
}

// K row groups of W lanes: in iteration j, group k runs stage 1 on row a0 + k, stage 2 on
// a0 + k - 1, stage 3 on a0 + k - 2 and stage 4 on a0 + k - 3, with a0 = y0 - 3 + j K, so an item of
// `chunk` rows takes (chunk + 6) / K iterations.  With K > 1 the moments (stage 1 -> 2) and the local
// transposes (stage 2 -> 3) of a row are made by one group and used by the next, so they go through
// LDS rings too; with K = 1 they stay in registers.  Every node runs the same arithmetic for every
// W and K.
template <typename T>
__device__ __forceinline__ Phys<T> adj_phys(const AdjArgs<T>& A);
template <>
__device__ __forceinline__ Phys<float> adj_phys<float>(const AdjArgs<float>& A)
{
    return A.Pf;
}
template <>
__device__ __forceinline__ Phys<double> adj_phys<double>(const AdjArgs<double>& A)
{
    return A.P;
}

template <typename T, int W, int K, int HOIST>
__global__ __launch_bounds__(W * K) void k_adj2d(AdjArgs<T> A)
{
    using C = T;  // arithmetic type: the storage type
    constexpr int R = K + 2;              // ring rows
    constexpr int RX = K > 1 ? R : 1;     // rings of moments and local transposes (K > 1 only)
    __shared__ C sC[R][3][W];  // dC_m of stage-1 rows
    __shared__ C sA[R][9][W];  // Gbar_{m,x}, Gbar_{m,y} (m-major), Lbar_m of stage-2 rows
    __shared__ C sS[R][5][W];  // S_f, J_x, J_y, S_g, S_k of stage-3 rows
    __shared__ C sM[RX][5][K > 1 ? W : 1];  // drho, jx, jy, phi, dpsi of stage-1 rows
    __shared__ C sL[RX][8][K > 1 ? W : 1];  // local-transpose outputs of stage-2 rows
    __shared__ double sred[3][W * K];

    const int item = xcd_item(blockIdx.x, gridDim.x);
    const int strip = item / A.nchunks, chunk = item - strip * A.nchunks;
    const int l = threadIdx.x % W;
    const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x / W);
    const int nx = A.nx, ny = A.ny;
    const int N = (int)A.N;
    const int x0 = strip * (W - 6);
    const int x = modi(x0 - 3 + l, nx);
    const int xm = wrapi(x - 1, nx), xp = wrapi(x + 1, nx);
    const bool own_x = l >= 3 && l < W - 3 && x0 + (l - 3) < nx;
    const int y0 = chunk * A.chunk;
    const int y1 = (y0 + A.chunk < ny) ? y0 + A.chunk : ny;
    const bool walls = A.walls != 0;
    const Phys<C> P = adj_phys<T>(A);
    const C w0 = C(weight<L9>(0));

    Moments<C> mom_prev = {};
    C lb_prev[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double kacc[3] = {0.0, 0.0, 0.0};
    // ring slot of row r (every row touched is >= y0 - 3)
    auto slot = [&](int r) { return (r - y0 + 3) % R; };
    // Global accesses are raw buffer accesses: one descriptor per 27 N array, a per-lane column
    // offset and a wavefront-uniform (scalar) offset for the species, direction and row.
    constexpr uint32_t ES = sizeof(T);
    const uint32_t nxu = (uint32_t)nx, Nu = (uint32_t)N, NB = Nu * ES;
    const Rsrc ru = make_rsrc(A.u, 27u * NB), rl1 = make_rsrc(A.lam1, 27u * NB), rl0 = make_rsrc(A.lam0, 27u * NB);
    const uint32_t vx0 = (uint32_t)x * ES, vxm = (uint32_t)xm * ES, vxp = (uint32_t)xp * ES;

    // stage 1 and stage 2 run on rows a and a - 1 of a group when these are inside the item's reach
    auto act12 = [&](int a_, bool& g1, bool& g2) {
        const int b_ = a_ - 1;
        const bool live_ = a_ < y1 + 3;
        g1 = live_ && (!walls || (a_ >= 0 && a_ < ny));
        g2 = live_ && b_ >= y0 - 2 && (!walls || (b_ >= 0 && b_ < ny)) && l >= 1 && l < W - 1;
    };
    // pull of row a_: direction i from r - e_i, or opp(i) at r where r - e_i lies beyond a wall
    auto load_pull = [&](int a_, T* pu) {
        const int row = (walls || (a_ >= 0 && a_ < ny)) ? a_ : modi(a_, ny);
        const uint32_t ym = row == 0 ? ny - 1 : row - 1, yp = row == ny - 1 ? 0 : row + 1;
        if (!walls || (row > 0 && row < ny - 1)) {
            // no wall next to the row: every direction pulls from r - e_i
            // source row offset by 1 - e_y: r - e_i lies in row ym for e_y = 1, row for 0, yp for -1
            const uint32_t ro[3] = {ym * nxu * ES, (uint32_t)row * nxu * ES, yp * nxu * ES};
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int ex = L9::ex[i], ey = L9::ey[i];
                const uint32_t so = (uint32_t)i * NB + ro[1 - ey];
                const uint32_t v = ex == 0 ? vx0 : (ex == 1 ? vxm : vxp);
                pu[i] = bload<T>(ru, v, so);
                pu[9 + i] = bload<T>(ru, v, so + 9u * NB);
                pu[18 + i] = bload<T>(ru, v, so + 18u * NB);
            }
            return;
        }
        const bool blo = walls && row == 0, bhi = walls && row == ny - 1;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int ex = L9::ex[i], ey = L9::ey[i];
            const bool bb = (ey == 1) ? blo : (ey == -1) ? bhi : false;
            const uint32_t ys = ey == 0 ? (uint32_t)row : (ey == 1 ? ym : yp);
            const uint32_t so = bb ? (uint32_t)L9::opp[i] * NB + (uint32_t)row * nxu * ES : (uint32_t)i * NB + ys * nxu * ES;
            const uint32_t v = bb ? vx0 : (ex == 0 ? vx0 : (ex == 1 ? vxm : vxp));
            pu[i] = bload<T>(ru, v, so);
            pu[9 + i] = bload<T>(ru, v, so + 9u * NB);
            pu[18 + i] = bload<T>(ru, v, so + 18u * NB);
        }
    };
    // lambda_{t+1} of row b_
    auto load_lam = [&](int b_, T* la) {
        const uint32_t so = (uint32_t)((walls || (b_ >= 0 && b_ < ny)) ? b_ : modi(b_, ny)) * nxu * ES;
#pragma unroll
        for (int q = 0; q < 27; ++q) la[q] = bload<T>(rl1, vx0, so + (uint32_t)q * NB);
    };
    // HOIST == 2: the pull and lambda_{t+1} rows of the next iteration are loaded during this one
    T pn[HOIST == 2 ? 27 : 1], ln[HOIST == 2 ? 27 : 1];
    if constexpr (HOIST == 2) {
        bool g1, g2;
        act12(y0 - 3 + grp, g1, g2);
        if (g1) load_pull(y0 - 3 + grp, pn);
        if (g2) load_lam(y0 - 4 + grp, ln);
    }

    for (int a0 = y0 - 3; a0 < y1 + 3; a0 += K) {
        const int a = a0 + grp, b = a - 1, c = a - 2, d = a - 3;
        const bool live = a < y1 + 3;
        bool act1, act2;
        act12(a, act1, act2);
        const bool act3 = live && c >= y0 - 1 && (!walls || (c >= 0 && c < ny)) && l >= 2 && l < W - 2;
        const bool act4 = live && d >= y0 && own_x;
        // ---- the global loads of the iteration come first: the pull of row a (stage 1), lambda_{t+1}
        // of row b (stage 2) and, with HOIST == 1, the gather of lambda_{t+1} around row d (stage 4), so
        // that none of them waits behind a store of stage 4 ----
        T pu[27], la[27], lg[27];
        // lambda_{t+1} around row d (d is a fluid row): direction j from r + e_j, or opp(j) at r where
        // r + e_j lies beyond a wall
        const bool d_in = !walls || (d > 0 && d < ny - 1);  // no wall next to row d
        auto gather = [&]() {
            const uint32_t dm = d == 0 ? ny - 1 : d - 1, dp = d == ny - 1 ? 0 : d + 1;
            if (d_in) {
                // source row offset by 1 + e_y: r + e_j lies in row dm for e_y = -1, d for 0, dp for 1
                const uint32_t ro[3] = {dm * nxu * ES, (uint32_t)d * nxu * ES, dp * nxu * ES};
#pragma unroll
                for (int j = 0; j < 9; ++j) {
                    const int ex = L9::ex[j], ey = L9::ey[j];
                    const uint32_t so = (uint32_t)j * NB + ro[1 + ey];
                    const uint32_t v = ex == 0 ? vx0 : (ex == 1 ? vxp : vxm);
                    lg[j] = bload<T>(rl1, v, so);
                    lg[9 + j] = bload<T>(rl1, v, so + 9u * NB);
                    lg[18 + j] = bload<T>(rl1, v, so + 18u * NB);
                }
                return;
            }
            const bool blo = walls && d == 0, bhi = walls && d == ny - 1;
#pragma unroll
            for (int j = 0; j < 9; ++j) {
                const int ex = L9::ex[j], ey = L9::ey[j];
                const bool bb = (ey == -1) ? blo : (ey == 1) ? bhi : false;
                const uint32_t yy = ey == 0 ? (uint32_t)d : (ey == 1 ? dp : dm);
                const uint32_t so = bb ? (uint32_t)L9::opp[j] * NB + (uint32_t)d * nxu * ES : (uint32_t)j * NB + yy * nxu * ES;
                const uint32_t v = bb ? vx0 : (ex == 0 ? vx0 : (ex == 1 ? vxp : vxm));
                lg[j] = bload<T>(rl1, v, so);
                lg[9 + j] = bload<T>(rl1, v, so + 9u * NB);
                lg[18 + j] = bload<T>(rl1, v, so + 18u * NB);
            }
        };
        if constexpr (HOIST == 2) {
#pragma unroll
            for (int q = 0; q < 27; ++q) {
                pu[q] = pn[q];
                la[q] = ln[q];
            }
        } else {
            if (act1) load_pull(a, pu);
            if (act2) load_lam(b, la);
        }
        if (HOIST == 1 && act4) gather();
        // ---- stage 1: moments and dC of row a ----
        Moments<C> mom_new = {};
        if (act1) {
            mom_new = moments_as<C, L9>(pu, pu + 9, pu + 18);
            C dc[3];
            conc_dev<C>(mom_new, dc);
            const int sa = slot(a);
#pragma unroll
            for (int m = 0; m < 3; ++m) sC[sa][m][l] = dc[m];
            if constexpr (K > 1) {
                sM[sa][0][l] = mom_new.drho;
                sM[sa][1][l] = mom_new.jx;
                sM[sa][2][l] = mom_new.jy;
                sM[sa][3][l] = mom_new.phi;
                sM[sa][4][l] = mom_new.dpsi;
            }
        }
        __syncthreads();
        // ---- stage 2: stencils and local transpose of row b = a - 1 ----
        C lb_new[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (act2) {
            const int s0 = slot(b), sm = slot(b - 1), sp = slot(a);
            if constexpr (K > 1) {
                mom_prev.drho = sM[s0][0][l];
                mom_prev.jx = sM[s0][1][l];
                mom_prev.jy = sM[s0][2][l];
                mom_prev.jz = C(0);
                mom_prev.phi = sM[s0][3][l];
                mom_prev.dpsi = sM[s0][4][l];
            }
            const bool glo = walls && b == 0, ghi = walls && b == ny - 1;
            C dc[3], gx[3], gy[3], lC[3];
            // gradients and Laplacian of C_m from its 3x3 neighbourhood v[dy+1][dx+1]
            auto stencil = [&](int m, const C (&v)[3][3]) {
                dc[m] = v[1][1];
                C sx = 0, sy = 0, lp = 0;
#pragma unroll
                for (int i = 1; i < 9; ++i) {
                    const C c = v[1 + L9::ey[i]][1 + L9::ex[i]];
                    const C w = C(weight<L9>(i));
                    sx += w * C(L9::ex[i]) * c;
                    sy += w * C(L9::ey[i]) * c;
                    lp += w * (c - dc[m]);
                }
                gx[m] = C(3) * sx;
                gy[m] = C(3) * sy;
                lC[m] = C(6) * lp;
            };
            if (!glo && !ghi) {
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    C v[3][3];
#pragma unroll
                    for (int dy = 0; dy < 3; ++dy) {
                        const int sr = dy == 0 ? sm : (dy == 1 ? s0 : sp);
                        v[dy][0] = sC[sr][m][l - 1];
                        v[dy][1] = sC[sr][m][l];
                        v[dy][2] = sC[sr][m][l + 1];
                    }
                    stencil(m, v);
                }
            } else {
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    C v[3][3];
                    v[1][0] = sC[s0][m][l - 1];
                    v[1][1] = sC[s0][m][l];
                    v[1][2] = sC[s0][m][l + 1];
                    if (glo) {  // ghost row below a lower wall
                        const T* wl = A.wet + m * nx;
                        v[0][0] = v[1][0] + C(wl[xm]);
                        v[0][1] = v[1][1] + C(wl[x]);
                        v[0][2] = v[1][2] + C(wl[xp]);
                    } else {
                        v[0][0] = sC[sm][m][l - 1];
                        v[0][1] = sC[sm][m][l];
                        v[0][2] = sC[sm][m][l + 1];
                    }
                    if (ghi) {  // ghost row above an upper wall
                        const T* wh = A.wet + (3 + m) * nx;
                        v[2][0] = v[1][0] + C(wh[xm]);
                        v[2][1] = v[1][1] + C(wh[x]);
                        v[2][2] = v[1][2] + C(wh[xp]);
                    } else {
                        v[2][0] = sC[sp][m][l - 1];
                        v[2][1] = sC[sp][m][l];
                        v[2][2] = sC[sp][m][l + 1];
                    }
                    stencil(m, v);
                }
            }
            C bG[3][2], bL[3], kb[3];
            adj_local<C, T>(P, mom_prev, dc, gx, gy, lC, la, lb_new, bG, bL, kb);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                sA[s0][2 * m][l] = bG[m][0];
                sA[s0][2 * m + 1][l] = bG[m][1];
                sA[s0][6 + m][l] = bL[m];
            }
            if constexpr (K > 1) {
#pragma unroll
                for (int q = 0; q < 8; ++q) sL[s0][q][l] = lb_new[q];
            }
            if (own_x && b >= y0 && b < y1) {
#pragma unroll
                for (int m = 0; m < 3; ++m) kacc[m] += (double)kb[m];
            }
        }
        // variant 2: the next iteration's pull and lambda rows, whose latency stages 3 and 4 cover
        if constexpr (HOIST == 2) {
            bool g1, g2;
            act12(a + K, g1, g2);
            if (g1) load_pull(a + K, pn);
            if (g2) load_lam(b + K, ln);
        }
        __syncthreads();
        // ---- stage 3: transposed stencils, ghost transposes, moment transpose of row c = a - 2 ----
        if (act3) {
            const int q0 = slot(c), qm = slot(c - 1), qp = slot(b);
            if constexpr (K > 1) {
#pragma unroll
                for (int q = 0; q < 8; ++q) lb_prev[q] = sL[q0][q][l];
            }
            C Cb[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) Cb[m] = lb_prev[5 + m] - C(6) * (C(1) - w0) * sA[q0][6 + m][l];
            // neighbour r - e_i of row c, skipped where it lies beyond a wall (a ghost, transposed below)
            auto tstencil = [&](int i) {
                const int ey = L9::ey[i], ex = L9::ex[i];
                const int sl = ey == 0 ? q0 : (ey == 1 ? qm : qp);  // row c - ey
                const int ln = l - ex;
                const C w = C(weight<L9>(i));
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    Cb[m] += C(3) * w * (C(ex) * sA[sl][2 * m][ln] + C(ey) * sA[sl][2 * m + 1][ln]) +
                             C(6) * w * sA[sl][6 + m][ln];
            };
            if (!walls || (c > 0 && c < ny - 1)) {
#pragma unroll
                for (int i = 1; i < 9; ++i) tstencil(i);
            } else {
#pragma unroll
                for (int i = 1; i < 9; ++i) {
                    const int ey = L9::ey[i];
                    if ((ey == 1 && c == 0) || (ey == -1 && c == ny - 1)) continue;
                    tstencil(i);
                }
            }
            if (walls && (c == 0 || c == ny - 1)) {
                const int wall = (c == 0) ? 0 : 1;
                const int side = (c == 0) ? -1 : 1;
                C Cg[3] = {0, 0, 0};
#pragma unroll
                for (int i = 1; i < 9; ++i) {
                    if (L9::ey[i] != side) continue;
                    const int ex = L9::ex[i], ey = L9::ey[i];
                    const int ln = l - ex;
                    const C w = C(weight<L9>(i));
#pragma unroll
                    for (int m = 0; m < 3; ++m)
                        Cg[m] += C(3) * w * (C(ex) * sA[q0][2 * m][ln] + C(ey) * sA[q0][2 * m + 1][ln]) +
                                 C(6) * w * sA[q0][6 + m][ln];
                }
                const bool own = own_x && c >= y0 && c < y1;
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    Cb[m] += Cg[m];
                    if (own) {
                        // C_ghost = C_adj + h / (alpha^2 kappa):  d/dh = 1/(alpha^2 kappa), d/dkappa = -wet / kappa
                        A.dh[(wall * 3 + m) * nx + x] += (double)Cg[m] / (double)P.a2kappa[m];
                        kacc[m] -= (double)Cg[m] * (double)A.wet[(wall * 3 + m) * nx + x] / (double)P.kappa[m];
                    }
                }
            }
            // transpose of C1 = (rho + phi - psi)/2, C2 = (rho - phi - psi)/2, C3 = psi
            sS[q0][0][l] = lb_prev[0] + C(0.5) * (Cb[0] + Cb[1]);
            sS[q0][1][l] = lb_prev[1];
            sS[q0][2][l] = lb_prev[2];
            sS[q0][3][l] = lb_prev[3] + C(0.5) * (Cb[0] - Cb[1]);
            sS[q0][4][l] = lb_prev[4] - C(0.5) * (Cb[0] + Cb[1]) + Cb[2];
        }
        __syncthreads();
        // ---- stage 4: lambda_t of row d = a - 3 from the gathered lambda_{t+1} and S, J ----
        if (act4) {
            if (HOIST != 1) gather();  // all 27 loads before the first store
            const int p0 = slot(d), pm = slot(d - 1), pp = slot(c);
            const uint32_t so = (uint32_t)d * nxu * ES;
            if (d_in) {
#pragma unroll
                for (int j = 0; j < 9; ++j) {
                    const int ln = l + L9::ex[j];
                    const int sl = L9::ey[j] == 0 ? p0 : (L9::ey[j] == 1 ? pp : pm);
                    const C Sf = sS[sl][0][ln], Jx = sS[sl][1][ln], Jy = sS[sl][2][ln];
                    const C Sg = sS[sl][3][ln], Sk = sS[sl][4][ln];
                    bstore<T>(T((C(1) - P.omega[0]) * C(lg[j]) + Sf + (C(L9::ex[j]) * Jx + C(L9::ey[j]) * Jy)), rl0,
                              vx0, so + (uint32_t)j * NB);
                    bstore<T>(T((C(1) - P.omega[1]) * C(lg[9 + j]) + Sg), rl0, vx0, so + (uint32_t)(9 + j) * NB);
                    bstore<T>(T((C(1) - P.omega[2]) * C(lg[18 + j]) + Sk), rl0, vx0, so + (uint32_t)(18 + j) * NB);
                }
            } else {
#pragma unroll
            for (int j = 0; j < 9; ++j) {
                const int yy = d + L9::ey[j];
                const bool bb = walls && (yy < 0 || yy >= ny);
                const int ln = bb ? l : l + L9::ex[j];
                const int sl = bb ? p0 : (L9::ey[j] == 0 ? p0 : (L9::ey[j] == 1 ? pp : pm));
                const C sgn = bb ? C(-1) : C(1);  // e of the gathered direction: e_j, or e_opp(j) = -e_j
                const C Sf = sS[sl][0][ln], Jx = sS[sl][1][ln], Jy = sS[sl][2][ln];
                const C Sg = sS[sl][3][ln], Sk = sS[sl][4][ln];
                bstore<T>(T((C(1) - P.omega[0]) * C(lg[j]) + Sf + sgn * (C(L9::ex[j]) * Jx + C(L9::ey[j]) * Jy)), rl0,
                          vx0, so + (uint32_t)j * NB);
                bstore<T>(T((C(1) - P.omega[1]) * C(lg[9 + j]) + Sg), rl0, vx0, so + (uint32_t)(9 + j) * NB);
                bstore<T>(T((C(1) - P.omega[2]) * C(lg[18 + j]) + Sk), rl0, vx0, so + (uint32_t)(18 + j) * NB);
            }
            }
        }
        if constexpr (K == 1) {
            mom_prev = mom_new;
#pragma unroll
            for (int q = 0; q < 8; ++q) lb_prev[q] = lb_new[q];
        }
    }
    // kappa gradient of the item: threads in a fixed tree
    const int t = threadIdx.x;
#pragma unroll
    for (int m = 0; m < 3; ++m) sred[m][t] = kacc[m];
    __syncthreads();
    for (int w = W * K / 2; w > 0; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int m = 0; m < 3; ++m) sred[m][t] += sred[m][t + w];
        }
        __syncthreads();
    }
    if (t < 3) {
        double* kp = A.kpart + t * A.nitems + item;
        *kp = A.kassign ? sred[t][0] : *kp + sred[t][0];
    }
}

// Inverse of the pull: position in u of the value that the pull of node (x, y) reads for direction i.
template <typename T>
__device__ __forceinline__ int64_t unstream(const AuxGeom& g, int i, int x, int y)
{
    const int ys = y - L9::ey[i];
    if (g.walls && (ys < 0 || ys >= g.ny)) return (int64_t)L9::opp[i] * g.N + (int64_t)y * g.nx + x;
    return (int64_t)i * g.N + (int64_t)wrapi(ys, g.ny) * g.nx + wrapi(x - L9::ex[i], g.nx);
}

// lambda_T from dL/dC_m of the state s_T: s_bar = (dC/ds)^T dL/dC, pushed through P^T.
template <typename T>
__global__ void k_adj_seed(AuxGeom g, const T* __restrict__ dC, T* __restrict__ lam)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const int x = (int)(n % g.nx), y = (int)(n / g.nx);
    const T g1 = dC ? dC[n] : T(0), g2 = dC ? dC[g.N + n] : T(0), g3 = dC ? dC[2 * g.N + n] : T(0);
    const T sf = T(0.5) * (g1 + g2), sg = T(0.5) * (g1 - g2), sk = T(-0.5) * (g1 + g2) + g3;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int64_t o = unstream<T>(g, i, x, y);
        lam[o] = sf;
        lam[9 * g.N + o] = sg;
        lam[18 * g.N + o] = sk;
    }
}

__global__ void k_fill0(double* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// Fixed-order reduction of the per-item kappa partials [3][n] into out[3] (+=): block m sums part[m][.]
// with each of its 256 threads taking a fixed strided subset in order, then a fixed tree.
__global__ __launch_bounds__(256) void k_reduce_items(const double* __restrict__ part, int64_t n,
                                                      double* __restrict__ out)
{
    __shared__ double red[256];
    const int m = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += part[m * n + i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[m] += red[0];
}

inline dim3 gridN(int64_t N) { return dim3((unsigned)((N + 255) / 256)); }

}  // namespace

template <typename T, int HOIST>
static bool launch_adj_w(const AdjArgs<T>& a, int width, int rows, hipStream_t s)
{
    const dim3 g(a.nitems);
    if (width == 64 && rows == 1) hipLaunchKernelGGL((k_adj2d<T, 64, 1, HOIST>), g, dim3(64), 0, s, a);
    else if (width == 64 && rows == 2) hipLaunchKernelGGL((k_adj2d<T, 64, 2, HOIST>), g, dim3(128), 0, s, a);
    else if (width == 64 && rows == 4) hipLaunchKernelGGL((k_adj2d<T, 64, 4, HOIST>), g, dim3(256), 0, s, a);
    else if (width == 128 && rows == 1) hipLaunchKernelGGL((k_adj2d<T, 128, 1, HOIST>), g, dim3(128), 0, s, a);
    else if (width == 128 && rows == 2) hipLaunchKernelGGL((k_adj2d<T, 128, 2, HOIST>), g, dim3(256), 0, s, a);
    else if (width == 256 && rows == 1) hipLaunchKernelGGL((k_adj2d<T, 256, 1, HOIST>), g, dim3(256), 0, s, a);
    else return false;
    return true;
}

template <typename T>
hipError_t launch_adjoint_sweep(const AdjArgs<T>& a, int width, int rows, int variant, hipStream_t s)
{
    const bool ok = variant == 2   ? launch_adj_w<T, 2>(a, width, rows, s)
                    : variant == 1 ? launch_adj_w<T, 1>(a, width, rows, s)
                                   : launch_adj_w<T, 0>(a, width, rows, s);
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_seed(const AuxGeom& g, const T* dC, T* lam, hipStream_t s)
{
    hipLaunchKernelGGL((k_adj_seed<T>), gridN(g.N), dim3(256), 0, s, g, dC, lam);
    return hipGetLastError();
}

hipError_t launch_fill0(double* p, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill0, gridN(n), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_reduce_items(const double* part, int64_t n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_items, dim3(3), dim3(256), 0, s, part, n, out);
    return hipGetLastError();
}

template hipError_t launch_adjoint_sweep<float>(const AdjArgs<float>&, int, int, int, hipStream_t);
template hipError_t launch_adjoint_sweep<double>(const AdjArgs<double>&, int, int, int, hipStream_t);
template hipError_t launch_adjoint_seed<float>(const AuxGeom&, const float*, float*, hipStream_t);
template hipError_t launch_adjoint_seed<double>(const AuxGeom&, const double*, double*, hipStream_t);

}  // namespace tlb
