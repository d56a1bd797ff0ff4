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
// Its transpose runs in three per-node passes:
//   1. moments and concentrations of s_t = P u_t                 (k_adj_fields)
//   2. the local transpose of E and of the relaxation: adjoints of the
//      moments, of C_m used locally, of G_m and L_m, and the direct kappa
//      terms                                                      (k_adj_local)
//   3. the transposed stencils  Cbar_m(r) += sum_i [3 w_i e_i . Gbar_m(r - e_i)
//      + 6 w_i Lbar_m(r - e_i)] - 6 (1 - w_0) Lbar_m(r), the transpose of the
//      ghost rows (hbar_m += Cbar_ghost / (alpha^2 kappa_m) and the kappa term
//      of the ghost value), the transpose of the moments, and the transpose of
//      P (a push through the inverse permutation)                 (k_adj_push)
// Per-node kappa contributions accumulate in an FP64 field that is reduced
// at the end, so every sum has a fixed order.
#include <stdint.h>

#include "../../include/tlb.h"
#include "tlb_internal.hpp"

namespace tlb {

namespace {

using L9 = D2Q9;

__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// Scratch layouts: F [8][N] = dC_m (3), drho, jx, jy, phi, dpsi;
// Abar [17][N] = drho_b, jx_b, jy_b, phi_b, dpsi_b, cbar_m (3), Gbar_{m,a} (6, m-major), Lbar_m (3).
constexpr int kF = 8, kA = 17;

template <typename T>
__global__ void k_adj_fields(AuxGeom g, const T* __restrict__ u, T* __restrict__ F)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const int x = (int)(n % g.nx), y = (int)(n / g.nx);
    T f[9], gg[9], k[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int ys = y - L9::ey[i];
        int64_t off;
        if (g.walls && (ys < 0 || ys >= g.ny))
            off = (int64_t)L9::opp[i] * g.N + n;
        else
            off = (int64_t)i * g.N + (int64_t)wrapi(ys, g.ny) * g.nx + wrapi(x - L9::ex[i], g.nx);
        f[i] = u[off];
        gg[i] = u[9 * g.N + off];
        k[i] = u[18 * g.N + off];
    }
    const Moments<T> mo = moments<L9, T>(f, gg, k);
    T dc[3];
    conc_dev<T>(mo, dc);
    F[0 * g.N + n] = dc[0];
    F[1 * g.N + n] = dc[1];
    F[2 * g.N + n] = dc[2];
    F[3 * g.N + n] = mo.drho;
    F[4 * g.N + n] = mo.jx;
    F[5 * g.N + n] = mo.jy;
    F[6 * g.N + n] = mo.phi;
    F[7 * g.N + n] = mo.dpsi;
}

// dC_m at neighbour (x + dx, y + dy) with the ghost rule beyond walls.
template <typename T>
__device__ __forceinline__ T dc_at(const AuxGeom& g, const T* F, const T* wet, int m, int x, int y)
{
    x = wrapi(x, g.nx);
    if (g.walls) {
        if (y < 0) return F[m * g.N + x] + wet[(0 * 3 + m) * g.nx + x];
        if (y >= g.ny) return F[m * g.N + (int64_t)(g.ny - 1) * g.nx + x] + wet[(1 * 3 + m) * g.nx + x];
    } else {
        y = wrapi(y, g.ny);
    }
    return F[m * g.N + (int64_t)y * g.nx + x];
}

template <typename T>
__global__ void k_adj_local(AuxGeom g, Phys<T> P, const T* __restrict__ F, const T* __restrict__ wet,
                            const T* __restrict__ lam1, T* __restrict__ Ab, double* __restrict__ kbar)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const int x = (int)(n % g.nx), y = (int)(n / g.nx);
    // forward quantities at the node
    T dc[3], gx[3], gy[3], lC[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        dc[m] = F[m * g.N + n];
        T sx = 0, sy = 0, lp = 0;
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const T c = dc_at<T>(g, F, wet, m, x + L9::ex[i], y + L9::ey[i]);
            const T w = T(weight<L9>(i));
            sx += w * T(L9::ex[i]) * c;
            sy += w * T(L9::ey[i]) * c;
            lp += w * (c - dc[m]);
        }
        gx[m] = T(3) * sx;
        gy[m] = T(3) * sy;
        lC[m] = T(6) * lp;
    }
    const T drho = F[3 * g.N + n], jx = F[4 * g.N + n], jy = F[5 * g.N + n];
    const T phi = F[6 * g.N + n], dpsi = F[7 * g.N + n];
    const T third = T(1.0 / 3.0);
    T c[3], mu[3];
    T pbx = drho * third, lam = 0, Txx = 0, Tyy = 0, Txy = 0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        c[m] = third + dc[m];
        mu[m] = P.kappa[m] * c[m] * (T(1) - c[m]) * (T(1) - T(2) * c[m]) - P.a2kappa[m] * lC[m];
        pbx += T(0.5) * P.kappa[m] * c[m] * c[m] * (T(1) - c[m]) * (T(1) - T(3) * c[m]);
        lam += P.a2kappa[m] * c[m] * lC[m];
        Txx += P.a2kappa[m] * gx[m] * gx[m];
        Tyy += P.a2kappa[m] * gy[m] * gy[m];
        Txy += P.a2kappa[m] * gx[m] * gy[m];
    }
    (void)mu;
    const T rho = T(1) + drho, irho = T(1) / rho;
    const T vx = jx * irho, vy = jy * irho, psi = third + dpsi, vv = vx * vx + vy * vy;

    // adjoint of the relaxation: Ebar = omega lambda'; rest populations from the mass constraints
    T af[9], ag[9], ak[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        af[i] = P.omega[0] * lam1[(int64_t)i * g.N + n];
        ag[i] = P.omega[1] * lam1[(int64_t)(9 + i) * g.N + n];
        ak[i] = P.omega[2] * lam1[(int64_t)(18 + i) * g.N + n];
    }
    T b_drho = af[0], b_phi = ag[0], b_dpsi = ak[0];
    T bA = 0, b_rho = 0, bBp = 0, bBk = 0, b_psi = 0, bTxx = 0, bTyy = 0, bTxy = 0, bvx = 0, bvy = 0, bvv = 0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const T w = T(weight<L9>(i));
        const T fb = af[i] - af[0], gb = ag[i] - ag[0], kb = ak[i] - ak[0];
        const T ev = T(L9::ex[i]) * vx + T(L9::ey[i]) * vy;
        const T U = T(3) * ev + T(4.5) * ev * ev - T(1.5) * vv;
        bA += w * fb;
        b_rho += w * U * fb;
        bTxx += T(3 * wdiag<L9>(i, 0)) * fb;
        bTyy += T(3 * wdiag<L9>(i, 1)) * fb;
        bTxy += T(3 * woff<L9>(i, 0, 1)) * fb;
        bBp += w * gb;
        b_phi += w * U * gb;
        bBk += w * kb;
        b_psi += w * U * kb;
        const T bU = w * (rho * fb + phi * gb + psi * kb);
        const T bev = bU * (T(3) + T(9) * ev);
        bvv += T(-1.5) * bU;
        bvx += T(L9::ex[i]) * bev;
        bvy += T(L9::ey[i]) * bev;
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
    T cbar[3], bG[3][2], bL[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const T cm = c[m];
        const T q = cm * (T(1) - cm) * (T(1) - T(2) * cm);
        const T dq = T(1) - T(6) * cm + T(6) * cm * cm;
        const T pp = cm * cm * (T(1) - cm) * (T(1) - T(3) * cm);
        const T dp = T(2) * cm - T(12) * cm * cm + T(12) * cm * cm * cm;
        cbar[m] = bmu[m] * P.kappa[m] * dq + b_pbx * T(0.5) * P.kappa[m] * dp + b_lam * P.a2kappa[m] * lC[m];
        bL[m] = -P.a2kappa[m] * bmu[m] + b_lam * P.a2kappa[m] * cm;
        bG[m][0] = bTxx * T(2) * P.a2kappa[m] * gx[m] + bTxy * P.a2kappa[m] * gy[m];
        bG[m][1] = bTyy * T(2) * P.a2kappa[m] * gy[m] + bTxy * P.a2kappa[m] * gx[m];
        const T kb = bmu[m] * (q - a2 * lC[m]) + b_pbx * T(0.5) * pp + b_lam * a2 * cm * lC[m] +
                     a2 * (bTxx * gx[m] * gx[m] + bTyy * gy[m] * gy[m] + bTxy * gx[m] * gy[m]);
        kbar[m * g.N + n] += (double)kb;
    }
    Ab[0 * g.N + n] = b_drho;
    Ab[1 * g.N + n] = b_jx;
    Ab[2 * g.N + n] = b_jy;
    Ab[3 * g.N + n] = b_phi;
    Ab[4 * g.N + n] = b_dpsi;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        Ab[(5 + m) * g.N + n] = cbar[m];
        Ab[(8 + 2 * m) * g.N + n] = bG[m][0];
        Ab[(9 + 2 * m) * g.N + n] = bG[m][1];
        Ab[(14 + m) * g.N + n] = bL[m];
    }
}

template <typename T>
__device__ __forceinline__ int64_t unstream(const AuxGeom& g, int i, int x, int y)
{
    const int ys = y - L9::ey[i];
    if (g.walls && (ys < 0 || ys >= g.ny)) return (int64_t)L9::opp[i] * g.N + (int64_t)y * g.nx + x;
    return (int64_t)i * g.N + (int64_t)wrapi(ys, g.ny) * g.nx + wrapi(x - L9::ex[i], g.nx);
}

template <typename T>
__global__ void k_adj_push(AuxGeom g, Phys<T> P, const T* __restrict__ Ab, const T* __restrict__ wet,
                           const T* __restrict__ lam1, T* __restrict__ lam0, double* __restrict__ dh,
                           double* __restrict__ kbar)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const int x = (int)(n % g.nx), y = (int)(n / g.nx);
    const T w0 = T(weight<L9>(0));
    T Cb[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) Cb[m] = Ab[(5 + m) * g.N + n] - T(6) * (T(1) - w0) * Ab[(14 + m) * g.N + n];
    // transposed stencils: contributions of the nodes r - e_i whose stencils read C(r)
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const int ys = y - L9::ey[i];
        if (g.walls && (ys < 0 || ys >= g.ny)) continue;
        const int64_t nn = (int64_t)wrapi(ys, g.ny) * g.nx + wrapi(x - L9::ex[i], g.nx);
        const T w = T(weight<L9>(i));
#pragma unroll
        for (int m = 0; m < 3; ++m)
            Cb[m] += T(3) * w * (T(L9::ex[i]) * Ab[(8 + 2 * m) * g.N + nn] + T(L9::ey[i]) * Ab[(9 + 2 * m) * g.N + nn]) +
                     T(6) * w * Ab[(14 + m) * g.N + nn];
    }
    // transposes of the ghost rows below / above this node (walls only)
    if (g.walls && (y == 0 || y == g.ny - 1)) {
        const int wall = (y == 0) ? 0 : 1;
        const int side = (y == 0) ? -1 : 1;  // e_y of the directions that reach the ghost row
        T Cg[3] = {0, 0, 0};
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            if (L9::ey[i] != side) continue;
            const int64_t nn = (int64_t)y * g.nx + wrapi(x - L9::ex[i], g.nx);
            const T w = T(weight<L9>(i));
#pragma unroll
            for (int m = 0; m < 3; ++m)
                Cg[m] += T(3) * w * (T(L9::ex[i]) * Ab[(8 + 2 * m) * g.N + nn] + T(L9::ey[i]) * Ab[(9 + 2 * m) * g.N + nn]) +
                         T(6) * w * Ab[(14 + m) * g.N + nn];
        }
        for (int m = 0; m < 3; ++m) {
            Cb[m] += Cg[m];
            // C_ghost = C_adj + h / (alpha^2 kappa):  d/dh = 1/(alpha^2 kappa), d/dkappa = -wet / kappa
            dh[(wall * 3 + m) * g.nx + x] += (double)Cg[m] / (double)P.a2kappa[m];
            kbar[m * g.N + n] -= (double)Cg[m] * (double)wet[(wall * 3 + m) * g.nx + x] / (double)P.kappa[m];
        }
    }
    // transpose of C1 = (rho + phi - psi)/2, C2 = (rho - phi - psi)/2, C3 = psi
    const T b_drho = Ab[0 * g.N + n] + T(0.5) * (Cb[0] + Cb[1]);
    const T b_jx = Ab[1 * g.N + n], b_jy = Ab[2 * g.N + n];
    const T b_phi = Ab[3 * g.N + n] + T(0.5) * (Cb[0] - Cb[1]);
    const T b_dpsi = Ab[4 * g.N + n] - T(0.5) * (Cb[0] + Cb[1]) + Cb[2];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int64_t o = unstream<T>(g, i, x, y);
        const T sf = (T(1) - P.omega[0]) * lam1[(int64_t)i * g.N + n] + b_drho + T(L9::ex[i]) * b_jx + T(L9::ey[i]) * b_jy;
        const T sg = (T(1) - P.omega[1]) * lam1[(int64_t)(9 + i) * g.N + n] + b_phi;
        const T sk = (T(1) - P.omega[2]) * lam1[(int64_t)(18 + i) * g.N + n] + b_dpsi;
        lam0[o] = sf;
        lam0[9 * g.N + o] = sg;
        lam0[18 * g.N + o] = sk;
    }
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

// Fixed-order reduction of the kappa field [3][N] into out[3] (+=) in two passes: kRedBlocks blocks per
// component sum fixed contiguous ranges into part[3][kRedBlocks], then one block per component sums those.
__device__ __forceinline__ double block_sum256(double v, double* red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

__global__ __launch_bounds__(256) void k_reduce3a(const double* __restrict__ f, int64_t N, double* __restrict__ part)
{
    __shared__ double red[256];
    const int m = blockIdx.x / kRedBlocks, j = blockIdx.x % kRedBlocks;
    const int64_t per = (N + kRedBlocks - 1) / kRedBlocks;
    const int64_t lo = j * per, hi = lo + per < N ? lo + per : N;
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) acc += f[m * N + i];
    const double t = block_sum256(acc, red);
    if (threadIdx.x == 0) part[m * kRedBlocks + j] = t;
}

__global__ __launch_bounds__(256) void k_reduce3b(const double* __restrict__ part, double* __restrict__ out)
{
    __shared__ double red[256];
    static_assert(kRedBlocks == 256, "one partial per lane");
    const double t = block_sum256(part[blockIdx.x * kRedBlocks + threadIdx.x], red);
    if (threadIdx.x == 0) out[blockIdx.x] += t;
}

inline dim3 gridN(int64_t N) { return dim3((unsigned)((N + 255) / 256)); }

}  // namespace

template <typename T>
hipError_t launch_adjoint_step(const AuxGeom& g, const Phys<T>& P, const T* u, const T* wet, const T* lam1, T* lam0,
                               T* F, T* Ab, double* dh, double* kbar, hipStream_t s)
{
    hipLaunchKernelGGL((k_adj_fields<T>), gridN(g.N), dim3(256), 0, s, g, u, F);
    hipLaunchKernelGGL((k_adj_local<T>), gridN(g.N), dim3(256), 0, s, g, P, F, wet, lam1, Ab, kbar);
    hipLaunchKernelGGL((k_adj_push<T>), gridN(g.N), dim3(256), 0, s, g, P, Ab, wet, lam1, lam0, dh, kbar);
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

hipError_t launch_reduce3(const double* f, int64_t N, double* part, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce3a, dim3(3 * kRedBlocks), dim3(256), 0, s, f, N, part);
    hipLaunchKernelGGL(k_reduce3b, dim3(3), dim3(256), 0, s, part, out);
    return hipGetLastError();
}

template hipError_t launch_adjoint_step<float>(const AuxGeom&, const Phys<float>&, const float*, const float*,
                                               const float*, float*, float*, float*, double*, double*, hipStream_t);
template hipError_t launch_adjoint_step<double>(const AuxGeom&, const Phys<double>&, const double*, const double*,
                                                const double*, double*, double*, double*, double*, double*,
                                                hipStream_t);
template hipError_t launch_adjoint_seed<float>(const AuxGeom&, const float*, float*, hipStream_t);
template hipError_t launch_adjoint_seed<double>(const AuxGeom&, const double*, double*, hipStream_t);

}  // namespace tlb
