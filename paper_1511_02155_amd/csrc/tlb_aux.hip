// Auxiliary kernels of the ternary LB library: initialisation to
// equilibrium, field readout, population import/export and the conservation
// check.  None of these is on the per-step hot path.
//
// The state buffer holds u_t (post-collision populations of the previous
// step, shifted storage); the post-propagation state s_t is its pull.
// Writing s_t into the buffer therefore uses the inverse of propagation,
// which with half-way bounce-back is a permutation: s_i(r) goes to
// u_i(r - e_i), or to u_opp(i)(r) when r - e_i is beyond a wall.
#include "tlb_internal.hpp"

namespace tlb {

namespace {

__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

__device__ __forceinline__ void node_xyz(const AuxGeom& g, int64_t n, int& x, int& y, int& z)
{
    x = (int)(n % g.nx);
    const int64_t r = n / g.nx;
    y = (int)(r % g.ny);
    z = (int)(r / g.ny);
}

__device__ __forceinline__ int64_t node_id(const AuxGeom& g, int x, int y, int z)
{
    return (int64_t)x + (int64_t)g.nx * ((int64_t)y + (int64_t)g.ny * z);
}

// Element of population j = s*Q + i of node (x, y, z) in a state: species-major [NC][Q][N] for D2Q9,
// plane-major blocks for D3Q19 (tlb_device.hpp).
template <class L, int NC>
__device__ __forceinline__ int64_t sidx(const AuxGeom& g, int j, int x, int y, int z)
{
    if constexpr (L::D == 2) {
        return (int64_t)j * g.N + node_id(g, x, y, z);
    } else {
        constexpr int NQ = NC * L::Q;
        return (int64_t)z * plane3d_elems(g.nx, g.ny, NQ) + plane3d_index(x + (int64_t)g.nx * y, NQ, j);
    }
}

// Pull of s_t at node (x, y, z) (generic lattice): p[NC][Q].
template <class L, int NC, typename T>
__device__ void pull_node(const AuxGeom& g, const T* __restrict__ st, int x, int y, int z, T* p)
{
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int ys = y - L::ey[i];
        const bool bb = g.walls && (ys < 0 || ys >= g.ny);
        const int ii = bb ? L::opp[i] : i;
        const int xs = bb ? x : wrapi(x - L::ex[i], g.nx);
        const int yy = bb ? y : wrapi(ys, g.ny);
        const int zs = bb ? z : wrapi(z - L::ez[i], g.nz);
#pragma unroll
        for (int s = 0; s < NC; ++s) p[s * L::Q + i] = st[sidx<L, NC>(g, s * L::Q + ii, xs, yy, zs)];
    }
}

// Element that receives s_i (species s) of node (x, y, z) under inverse propagation.
template <class L, int NC>
__device__ __forceinline__ int64_t unstream_idx(const AuxGeom& g, int s, int i, int x, int y, int z)
{
    const int ys = y - L::ey[i];
    if (g.walls && (ys < 0 || ys >= g.ny)) return sidx<L, NC>(g, s * L::Q + L::opp[i], x, y, z);
    return sidx<L, NC>(g, s * L::Q + i, wrapi(x - L::ex[i], g.nx), wrapi(ys, g.ny), wrapi(z - L::ez[i], g.nz));
}

// dC_m at a (possibly ghost) neighbour, read from an [nc][N] array of
// concentrations C (offset removed) with the wetting ghost rule; wet is [2][nc][nx*nz].
template <typename T, typename TIn, typename TW>
__device__ __forceinline__ T conc_at(const AuxGeom& g, const TIn* C, T offset, const TW* wet, int m, int x, int y,
                                     int z)
{
    x = wrapi(x, g.nx);
    z = wrapi(z, g.nz);
    const int64_t nxz = (int64_t)g.nx * g.nz;
    if (g.walls) {
        if (y < 0)
            return T(C[m * g.N + node_id(g, x, 0, z)]) - offset + T(wet[(0 * g.nc + m) * nxz + x + (int64_t)g.nx * z]);
        if (y >= g.ny)
            return T(C[m * g.N + node_id(g, x, g.ny - 1, z)]) - offset +
                   T(wet[(1 * g.nc + m) * nxz + x + (int64_t)g.nx * z]);
    } else {
        y = wrapi(y, g.ny);
    }
    return T(C[m * g.N + node_id(g, x, y, z)]) - offset;
}

// Isotropic stencils d_a X = 3 sum_i w_i e_ia X(r+e_i), lap X = 6 sum_i w_i [X(r+e_i) - X(r)].
template <class L, int NC, typename T, typename TIn, typename TW>
__device__ void stencil_at(const AuxGeom& g, const TIn* C, T offset, const TW* wet, int x, int y, int z, T dc[NC],
                           T gC[NC][3], T lC[NC])
{
#pragma unroll
    for (int m = 0; m < NC; ++m) {
        dc[m] = conc_at<T, TIn, TW>(g, C, offset, wet, m, x, y, z);
        T gx = 0, gy = 0, gz = 0, lp = 0;
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            const T c = conc_at<T, TIn, TW>(g, C, offset, wet, m, x + L::ex[i], y + L::ey[i], z + L::ez[i]);
            const T w = T(weight<L>(i));
            gx += w * T(L::ex[i]) * c;
            gy += w * T(L::ey[i]) * c;
            gz += w * T(L::ez[i]) * c;
            lp += w * (c - dc[m]);
        }
        gC[m][0] = T(3) * gx;
        gC[m][1] = T(3) * gy;
        gC[m][2] = T(3) * gz;
        lC[m] = T(6) * lp;
    }
}

template <class L, int NC, typename T, typename TIn>
__global__ void k_init(AuxGeom g, Phys<acc_t<T>> P, const TIn* __restrict__ C, const TIn* __restrict__ u,
                       const T* __restrict__ wet, T* __restrict__ st)
{
    using A = acc_t<T>;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    node_xyz(g, n, x, y, z);
    A dc[NC], gC[NC][3], lC[NC];
    stencil_at<L, NC, A, TIn, T>(g, C, A(psi_ref<NC>()), wet, x, y, z, dc, gC, lC);
    Moments<A, NC> mo;
    // rho = sum_m C_m, phi = C1 - C2, psi_l = C_l (Sec. II.C, II.E), as deviations
    mo.drho = dc[0];
#pragma unroll
    for (int m = 1; m < NC; ++m) mo.drho += dc[m];
    mo.phi = dc[0] - dc[1];
    mo.dpsi = dc[2];
#pragma unroll
    for (int l = 0; l < NC - 3; ++l) mo.dpsx[l] = dc[3 + l];
    const A rho = A(1) + mo.drho;
    mo.jx = u ? rho * A(u[n]) : A(0);
    mo.jy = u ? rho * A(u[g.N + n]) : A(0);
    mo.jz = (u && L::D == 3) ? rho * A(u[2 * g.N + n]) : A(0);
    T p[NC * L::Q];
    equilibrium<L, NC>(P, mo, dc, gC, lC, p, p + L::Q, p + 2 * L::Q);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
#pragma unroll
        for (int s = 0; s < NC; ++s) st[unstream_idx<L, NC>(g, s, i, x, y, z)] = p[s * L::Q + i];
    }
}

// Field rows (deviations): dC_m in rows 0 .. NC-1, then drho, phi, dpsi_3, ux, uy, uz, mu_phi, mu_psi
// (of psi_3).  For NC = 3 these are the TLB_FIELD_* selectors in order.
// Phase 1 of the readout: moments of s_t -> every row but the chemical potentials.
template <class L, int NC, typename T>
__global__ void k_fields1(AuxGeom g, const T* __restrict__ st, T* __restrict__ F)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    node_xyz(g, n, x, y, z);
    using A = acc_t<T>;
    T p[NC * L::Q];
    pull_node<L, NC, T>(g, st, x, y, z, p);
    const Moments<A, NC> mo = moments<L, NC>(p, p + L::Q, p + 2 * L::Q);
    A dc[NC];
    conc_dev<A, NC>(mo, dc);
    const A irho = A(1) / (A(1) + mo.drho);
#pragma unroll
    for (int m = 0; m < NC; ++m) F[m * g.N + n] = T(dc[m]);
    F[(NC + 0) * g.N + n] = T(mo.drho);
    F[(NC + 1) * g.N + n] = T(mo.phi);
    F[(NC + 2) * g.N + n] = T(mo.dpsi);
    F[(NC + 3) * g.N + n] = T(mo.jx * irho);
    F[(NC + 4) * g.N + n] = T(mo.jy * irho);
    F[(NC + 5) * g.N + n] = (L::D == 3) ? T(mo.jz * irho) : T(0);
}

// Phase 2: chemical potentials from the dC fields with the ghost rule.
template <class L, int NC, typename T>
__global__ void k_fields2(AuxGeom g, Phys<acc_t<T>> P, const T* __restrict__ wet, T* __restrict__ F)
{
    using A = acc_t<T>;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    node_xyz(g, n, x, y, z);
    A dc[NC], gC[NC][3], lC[NC];
    stencil_at<L, NC, A, T, T>(g, F, A(0), wet, x, y, z, dc, gC, lC);
    A mphi, mpsi;
    chem_potentials<A, NC>(P, dc, lC, mphi, mpsi);
    F[(NC + 6) * g.N + n] = T(mphi);
    F[(NC + 7) * g.N + n] = T(mpsi);
}

template <typename T, typename TOut>
__global__ void k_export(int64_t N, const T* __restrict__ src, T offset, TOut* __restrict__ out)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) out[n] = TOut(src[n]) + TOut(offset);
}

template <class L, int NC, typename T, typename TOut>
__global__ void k_get_pops(AuxGeom g, const T* __restrict__ st, int s, TOut* __restrict__ out)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    node_xyz(g, n, x, y, z);
    T p[NC * L::Q];
    pull_node<L, NC, T>(g, st, x, y, z, p);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) out[(int64_t)i * g.N + n] = TOut(p[s * L::Q + i]) + TOut(ref<L, NC>(s, i));
}

template <class L, int NC, typename T, typename TIn>
__global__ void k_set_pops(AuxGeom g, const TIn* __restrict__ in, int s, T* __restrict__ st)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    node_xyz(g, n, x, y, z);
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        st[unstream_idx<L, NC>(g, s, i, x, y, z)] = T(in[(int64_t)i * g.N + n]) - T(ref<L, NC>(s, i));
}

// Diagnostic slots (diag_slots(NC) of them): mass of rho, phi, psi_3 (0-2), momentum (3-5), max |v|
// (6, a maximum), the non-finite count (7), the interface sums of C1 .. C3 (8-10), then for NC > 3 the
// masses of psi_4 .. psi_NC and the interface sums of C4 .. C_NC.
//
// Block-level sums in FP64 with a fixed assignment of nodes to blocks (deterministic).
//
// Reduction of a 256-lane block: each wavefront folds its 64 lanes with a
// butterfly of cross-lane exchanges (5 xor steps of 32 .. 1 lanes, no LDS and
// no barrier), lane 0 of each of the four wavefronts writes its result to
// LDS, and after one barrier thread q adds (or takes the maximum of) the four
// wavefront results of slot q in wavefront order; red[q][0] then holds slot
// q.  Slot 6 is a maximum, the others sums.  The order is fixed, so results
// are reproducible bit for bit.
template <int S>
__device__ __forceinline__ void block_reduce(double (&acc)[S], double (&red)[S][4])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < S; ++q) {
        double v = acc[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double w = __shfl_xor(v, o, 64);
            v = (q == 6) ? fmax(v, w) : v + w;
        }
        if (lane == 0) red[q][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < S) {
        const int q = threadIdx.x;
        double v = red[q][0];
        for (int k = 1; k < 4; ++k) v = (q == 6) ? fmax(v, red[q][k]) : v + red[q][k];
        red[q][0] = v;
    }
}

template <class L, int NC, typename T>
__global__ __launch_bounds__(256) void k_diag1(AuxGeom g, const T* __restrict__ st, double* __restrict__ partial)
{
    constexpr int S = diag_slots(NC);
    __shared__ double red[S][4];
    double acc[S];
#pragma unroll
    for (int q = 0; q < S; ++q) acc[q] = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < g.N; n += (int64_t)gridDim.x * 256) {
        int x, y, z;
        node_xyz(g, n, x, y, z);
        T p[NC * L::Q];
        pull_node<L, NC, T>(g, st, x, y, z, p);
        const auto mo = moments<L, NC>(p, p + L::Q, p + 2 * L::Q);
        const double rho = 1.0 + (double)mo.drho;
        const double jx = mo.jx, jy = mo.jy, jz = mo.jz;
        double psi[NC - 2];
        psi[0] = psi_ref<NC>() + (double)mo.dpsi;
        bool finite = isfinite(rho) && isfinite(jx) && isfinite(jy) && isfinite(jz) && isfinite((double)mo.phi) &&
                      isfinite(psi[0]);
        double spsi = psi[0];
#pragma unroll
        for (int l = 1; l < NC - 2; ++l) {
            psi[l] = psi_ref<NC>() + (double)mo.dpsx[l - 1];
            finite = finite && isfinite(psi[l]);
            spsi += psi[l];
        }
        const double phi = mo.phi;
        if (finite) {
            acc[0] += rho;
            acc[1] += phi;
            acc[2] += psi[0];
            acc[3] += jx;
            acc[4] += jy;
            acc[5] += jz;
            const double sp = sqrt(jx * jx + jy * jy + jz * jz) / rho;
            acc[6] = fmax(acc[6], sp);
            // interface measure: C_m^2 (1 - C_m)^2 with C1 = (rho + phi - sum psi)/2,
            // C2 = (rho - phi - sum psi)/2, C_l = psi_l
            double c[NC];
            c[0] = 0.5 * (rho + phi - spsi);
            c[1] = 0.5 * (rho - phi - spsi);
#pragma unroll
            for (int l = 0; l < NC - 2; ++l) c[2 + l] = psi[l];
#pragma unroll
            for (int m = 0; m < 3; ++m) acc[8 + m] += c[m] * c[m] * (1.0 - c[m]) * (1.0 - c[m]);
#pragma unroll
            for (int l = 0; l < NC - 3; ++l) {
                acc[11 + l] += psi[1 + l];
                acc[11 + (NC - 3) + l] += c[3 + l] * c[3 + l] * (1.0 - c[3 + l]) * (1.0 - c[3 + l]);
            }
        } else {
            acc[7] += 1.0;
        }
    }
    block_reduce<S>(acc, red);
    if (threadIdx.x < S) partial[(int64_t)blockIdx.x * S + threadIdx.x] = red[threadIdx.x][0];
}

template <int S>
__global__ __launch_bounds__(256) void k_diag2(const double* __restrict__ partial, int nblocks, double* __restrict__ out)
{
    __shared__ double red[S][4];
    double acc[S];
#pragma unroll
    for (int q = 0; q < S; ++q) acc[q] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) {
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const double v = partial[(int64_t)b * S + q];
            acc[q] = (q == 6) ? fmax(acc[q], v) : acc[q] + v;
        }
    }
    block_reduce<S>(acc, red);
    if (threadIdx.x < S) out[threadIdx.x] = red[threadIdx.x][0];
}

// wet[m][j] = h[m][j] / (alpha^2 kappa_m) for the nc components of one wall.
template <typename T, typename TIn>
__global__ void k_wet(int n, int nc, const TIn* __restrict__ h, WetScale inv, T* __restrict__ wet)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nc * n) return;
    const int m = j / n;
    wet[j] = T((double)h[j] * inv.v[m]);
}

inline dim3 grid_for(int64_t N, int bs) { return dim3((unsigned)((N + bs - 1) / bs)); }

// One 16-byte vector per lane and one short-lived workgroup per 4 KiB: the
// form that reaches the highest copy bandwidth measured on MI355X.
template <typename TIn, typename TOut>
__global__ void k_convert(const TIn* __restrict__ in, TOut* __restrict__ out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = TOut(in[i]);
}

__global__ __launch_bounds__(256) void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace

template <typename TIn, typename TOut>
hipError_t launch_convert(const TIn* in, TOut* out, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL((k_convert<TIn, TOut>), grid_for(n, 256), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}
template hipError_t launch_convert<float, double>(const float*, double*, int64_t, hipStream_t);
template hipError_t launch_convert<double, double>(const double*, double*, int64_t, hipStream_t);

hipError_t launch_copy16(const void* src, void* dst, int64_t n16, hipStream_t s)
{
    const int64_t blocks = (n16 + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s, (const uint4*)src, (uint4*)dst, n16);
    return hipGetLastError();
}

// Dispatch on the lattice and the number of components (3, 4 or 5).
#define TLB_AUX_DISPATCH(KERNEL, GRID, BLOCK, S, ...)                                                       \
    do {                                                                                                  \
        if (g.lattice == 1 && g.nc == 3)                                                                  \
            hipLaunchKernelGGL((KERNEL<D3Q19, 3, __VA_ARGS__>), GRID, BLOCK, 0, S, ARGS);                  \
        else if (g.lattice == 1 && g.nc == 4)                                                             \
            hipLaunchKernelGGL((KERNEL<D3Q19, 4, __VA_ARGS__>), GRID, BLOCK, 0, S, ARGS);                  \
        else if (g.lattice == 1)                                                                          \
            hipLaunchKernelGGL((KERNEL<D3Q19, 5, __VA_ARGS__>), GRID, BLOCK, 0, S, ARGS);                  \
        else if (g.nc == 3)                                                                               \
            hipLaunchKernelGGL((KERNEL<D2Q9, 3, __VA_ARGS__>), GRID, BLOCK, 0, S, ARGS);                   \
        else if (g.nc == 4)                                                                               \
            hipLaunchKernelGGL((KERNEL<D2Q9, 4, __VA_ARGS__>), GRID, BLOCK, 0, S, ARGS);                   \
        else                                                                                              \
            hipLaunchKernelGGL((KERNEL<D2Q9, 5, __VA_ARGS__>), GRID, BLOCK, 0, S, ARGS);                   \
    } while (0)

template <typename T, typename TIn>
hipError_t launch_init(const AuxGeom& g, const Phys<acc_t<T>>& P, const TIn* C, const TIn* u, const T* wet, T* state,
                       hipStream_t s)
{
#define ARGS g, P, C, u, wet, state
    TLB_AUX_DISPATCH(k_init, grid_for(g.N, 256), dim3(256), s, T, TIn);
#undef ARGS
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fields(const AuxGeom& g, const Phys<acc_t<T>>& P, const T* state, const T* wet, T* F,
                         hipStream_t s)
{
#define ARGS g, state, F
    TLB_AUX_DISPATCH(k_fields1, grid_for(g.N, 256), dim3(256), s, T);
#undef ARGS
#define ARGS g, P, wet, F
    TLB_AUX_DISPATCH(k_fields2, grid_for(g.N, 256), dim3(256), s, T);
#undef ARGS
    return hipGetLastError();
}

int field_row(int nc, int which)
{
    if (which >= 0 && which <= 2) return which;        // C1 .. C3
    if (which >= 3 && which <= 10) return nc + which - 3;  // rho .. mu_psi
    if (which >= 11 && which < 11 + nc - 3) return which - 8;  // C4 .. C_nc
    return -1;
}

template <typename T, typename TOut>
hipError_t launch_export_field(const AuxGeom& g, const T* F, int which, TOut* out, hipStream_t s)
{
    const int row = field_row(g.nc, which);
    if (row < 0) return hipErrorInvalidValue;
    // offsets of the stored deviations: C_m and psi_3: 1/nc; rho: 1
    T off = 0;
    if (row < g.nc || which == 5) off = T(1.0 / g.nc);
    if (which == 3) off = T(1);
    hipLaunchKernelGGL((k_export<T, TOut>), grid_for(g.N, 256), dim3(256), 0, s, g.N, F + (int64_t)row * g.N, off,
                       out);
    return hipGetLastError();
}

template <typename T, typename TOut>
hipError_t launch_get_pops(const AuxGeom& g, const T* state, int species, TOut* out, hipStream_t s)
{
#define ARGS g, state, species, out
    TLB_AUX_DISPATCH(k_get_pops, grid_for(g.N, 256), dim3(256), s, T, TOut);
#undef ARGS
    return hipGetLastError();
}

template <typename T, typename TIn>
hipError_t launch_set_pops(const AuxGeom& g, const TIn* in, int species, T* state, hipStream_t s)
{
#define ARGS g, in, species, state
    TLB_AUX_DISPATCH(k_set_pops, grid_for(g.N, 256), dim3(256), s, T, TIn);
#undef ARGS
    return hipGetLastError();
}

template <typename T>
hipError_t launch_diag(const AuxGeom& g, const T* state, double* partial, int nblocks, double* out, hipStream_t s)
{
#define ARGS g, state, partial
    TLB_AUX_DISPATCH(k_diag1, dim3(nblocks), dim3(256), s, T);
#undef ARGS
    if (g.nc == 3)
        hipLaunchKernelGGL(k_diag2<diag_slots(3)>, dim3(1), dim3(256), 0, s, partial, nblocks, out);
    else if (g.nc == 4)
        hipLaunchKernelGGL(k_diag2<diag_slots(4)>, dim3(1), dim3(256), 0, s, partial, nblocks, out);
    else
        hipLaunchKernelGGL(k_diag2<diag_slots(5)>, dim3(1), dim3(256), 0, s, partial, nblocks, out);
    return hipGetLastError();
}
#undef TLB_AUX_DISPATCH

template <typename T, typename TIn>
hipError_t launch_wet(int n, int nc, const TIn* h, const WetScale& inv, T* wet, hipStream_t s)
{
    hipLaunchKernelGGL((k_wet<T, TIn>), grid_for((int64_t)nc * n, 256), dim3(256), 0, s, n, nc, h, inv, wet);
    return hipGetLastError();
}

#define TLB_INST_IO(T, TIO)                                                                                   \
    template hipError_t launch_init<T, TIO>(const AuxGeom&, const Phys<acc_t<T>>&, const TIO*, const TIO*,       \
                                            const T*, T*, hipStream_t);                                         \
    template hipError_t launch_export_field<T, TIO>(const AuxGeom&, const T*, int, TIO*, hipStream_t);            \
    template hipError_t launch_get_pops<T, TIO>(const AuxGeom&, const T*, int, TIO*, hipStream_t);                \
    template hipError_t launch_set_pops<T, TIO>(const AuxGeom&, const TIO*, int, T*, hipStream_t);                \
    template hipError_t launch_wet<T, TIO>(int, int, const TIO*, const WetScale&, T*, hipStream_t);

#define TLB_INST(T)                                                                                           \
    template hipError_t launch_fields<T>(const AuxGeom&, const Phys<acc_t<T>>&, const T*, const T*, T*,       \
                                         hipStream_t);                                                          \
    template hipError_t launch_diag<T>(const AuxGeom&, const T*, double*, int, double*, hipStream_t);

TLB_INST(float)
TLB_INST(double)
TLB_INST_IO(float, double)
TLB_INST_IO(float, float)
TLB_INST_IO(double, double)

}  // namespace tlb
