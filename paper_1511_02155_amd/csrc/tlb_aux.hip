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

// Pull of s_t at node (x, y, z) (generic lattice).
template <class L, typename T>
__device__ void pull_node(const AuxGeom& g, const T* __restrict__ st, int x, int y, int z, T* f, T* gg, T* k)
{
    const int64_t n0 = node_id(g, x, y, z);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int ys = y - L::ey[i];
        int64_t off;
        if (g.walls && (ys < 0 || ys >= g.ny)) {
            off = (int64_t)L::opp[i] * g.N + n0;
        } else {
            off = (int64_t)i * g.N + node_id(g, wrapi(x - L::ex[i], g.nx), wrapi(ys, g.ny), wrapi(z - L::ez[i], g.nz));
        }
        f[i] = st[off];
        gg[i] = st[(int64_t)L::Q * g.N + off];
        k[i] = st[(int64_t)2 * L::Q * g.N + off];
    }
}

// Inverse propagation target of direction i from node (x, y, z).
template <class L>
__device__ __forceinline__ int64_t unstream_off(const AuxGeom& g, int i, int x, int y, int z)
{
    const int ys = y - L::ey[i];
    if (g.walls && (ys < 0 || ys >= g.ny)) return (int64_t)L::opp[i] * g.N + node_id(g, x, y, z);
    return (int64_t)i * g.N + node_id(g, wrapi(x - L::ex[i], g.nx), wrapi(ys, g.ny), wrapi(z - L::ez[i], g.nz));
}

// dC_m at a (possibly ghost) neighbour, read from a [3][N] array of
// concentrations C (offset 1/3 removed) with the wetting ghost rule.
template <typename T, typename TIn, typename TW>
__device__ __forceinline__ T conc_at(const AuxGeom& g, const TIn* C, T offset, const TW* wet, int m, int x, int y,
                                     int z)
{
    x = wrapi(x, g.nx);
    z = wrapi(z, g.nz);
    const int64_t nxz = (int64_t)g.nx * g.nz;
    if (g.walls) {
        if (y < 0)
            return T(C[m * g.N + node_id(g, x, 0, z)]) - offset + T(wet[(0 * 3 + m) * nxz + x + (int64_t)g.nx * z]);
        if (y >= g.ny)
            return T(C[m * g.N + node_id(g, x, g.ny - 1, z)]) - offset +
                   T(wet[(1 * 3 + m) * nxz + x + (int64_t)g.nx * z]);
    } else {
        y = wrapi(y, g.ny);
    }
    return T(C[m * g.N + node_id(g, x, y, z)]) - offset;
}

// Isotropic stencils d_a X = 3 sum_i w_i e_ia X(r+e_i), lap X = 6 sum_i w_i [X(r+e_i) - X(r)].
template <class L, typename T, typename TIn, typename TW>
__device__ void stencil_at(const AuxGeom& g, const TIn* C, T offset, const TW* wet, int x, int y, int z, T dc[3],
                           T gC[3][3], T lC[3])
{
#pragma unroll
    for (int m = 0; m < 3; ++m) {
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

template <class L, typename T, typename TIn>
__global__ void k_init(AuxGeom g, Phys<acc_t<T>> P, const TIn* __restrict__ C, const TIn* __restrict__ u,
                       const T* __restrict__ wet, T* __restrict__ st)
{
    using A = acc_t<T>;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    node_xyz(g, n, x, y, z);
    A dc[3], gC[3][3], lC[3];
    stencil_at<L, A, TIn, T>(g, C, A(1.0 / 3.0), wet, x, y, z, dc, gC, lC);
    Moments<A> mo;
    // rho = C1 + C2 + C3, phi = C1 - C2, psi = C3 (Sec. II.C), as deviations
    mo.drho = dc[0] + dc[1] + dc[2];
    mo.phi = dc[0] - dc[1];
    mo.dpsi = dc[2];
    const A rho = A(1) + mo.drho;
    mo.jx = u ? rho * A(u[n]) : A(0);
    mo.jy = u ? rho * A(u[g.N + n]) : A(0);
    mo.jz = (u && L::D == 3) ? rho * A(u[2 * g.N + n]) : A(0);
    T f[L::Q], gg[L::Q], k[L::Q];
    equilibrium<L>(P, mo, dc, gC, lC, f, gg, k);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const int64_t off = unstream_off<L>(g, i, x, y, z);
        st[off] = f[i];
        st[(int64_t)L::Q * g.N + off] = gg[i];
        st[(int64_t)2 * L::Q * g.N + off] = k[i];
    }
}

// Phase 1 of the readout: moments of s_t -> fields [0..8] (deviations).
template <class L, typename T>
__global__ void k_fields1(AuxGeom g, const T* __restrict__ st, T* __restrict__ F)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    node_xyz(g, n, x, y, z);
    using A = acc_t<T>;
    T f[L::Q], gg[L::Q], k[L::Q];
    pull_node<L, T>(g, st, x, y, z, f, gg, k);
    const Moments<A> mo = moments<L, T>(f, gg, k);
    A dc[3];
    conc_dev<A>(mo, dc);
    const A irho = A(1) / (A(1) + mo.drho);
    F[0 * g.N + n] = T(dc[0]);
    F[1 * g.N + n] = T(dc[1]);
    F[2 * g.N + n] = T(dc[2]);
    F[3 * g.N + n] = T(mo.drho);
    F[4 * g.N + n] = T(mo.phi);
    F[5 * g.N + n] = T(mo.dpsi);
    F[6 * g.N + n] = T(mo.jx * irho);
    F[7 * g.N + n] = T(mo.jy * irho);
    F[8 * g.N + n] = (L::D == 3) ? T(mo.jz * irho) : T(0);
}

// Phase 2: chemical potentials from the dC fields with the ghost rule.
template <class L, typename T>
__global__ void k_fields2(AuxGeom g, Phys<acc_t<T>> P, const T* __restrict__ wet, T* __restrict__ F)
{
    using A = acc_t<T>;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    node_xyz(g, n, x, y, z);
    A dc[3], gC[3][3], lC[3];
    stencil_at<L, A, T, T>(g, F, A(0), wet, x, y, z, dc, gC, lC);
    A mphi, mpsi;
    chem_potentials<A>(P, dc, lC, mphi, mpsi);
    F[9 * g.N + n] = T(mphi);
    F[10 * g.N + n] = T(mpsi);
}

template <typename T, typename TOut>
__global__ void k_export(int64_t N, const T* __restrict__ src, T offset, TOut* __restrict__ out)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) out[n] = TOut(src[n]) + TOut(offset);
}

template <class L, typename T, typename TOut>
__global__ void k_get_pops(AuxGeom g, const T* __restrict__ st, int s, TOut* __restrict__ out)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    node_xyz(g, n, x, y, z);
    T f[L::Q], gg[L::Q], k[L::Q];
    pull_node<L, T>(g, st, x, y, z, f, gg, k);
    const T* v = (s == 0) ? f : (s == 1) ? gg : k;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) out[(int64_t)i * g.N + n] = TOut(v[i]) + TOut(ref<L>(s, i));
}

template <class L, typename T, typename TIn>
__global__ void k_set_pops(AuxGeom g, const TIn* __restrict__ in, int s, T* __restrict__ st)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    node_xyz(g, n, x, y, z);
    T* base = st + (int64_t)s * L::Q * g.N;
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        base[unstream_off<L>(g, i, x, y, z)] = T(in[(int64_t)i * g.N + n]) - T(ref<L>(s, i));
}

// Block-level sums of mass, momentum, max |v| and the non-finite count, in
// FP64, with a fixed assignment of nodes to blocks (deterministic).
template <class L, typename T>
__global__ __launch_bounds__(256) void k_diag1(AuxGeom g, const T* __restrict__ st, double* __restrict__ partial)
{
    __shared__ double red[kDiagSlots][256];
    double acc[kDiagSlots] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < g.N; n += (int64_t)gridDim.x * 256) {
        int x, y, z;
        node_xyz(g, n, x, y, z);
        T f[L::Q], gg[L::Q], k[L::Q];
        pull_node<L, T>(g, st, x, y, z, f, gg, k);
        const auto mo = moments<L, T>(f, gg, k);
        const double rho = 1.0 + (double)mo.drho;
        const double jx = mo.jx, jy = mo.jy, jz = mo.jz;
        const double phi = mo.phi, psi = kPsiRef + (double)mo.dpsi;
        const bool finite = isfinite(rho) && isfinite(jx) && isfinite(jy) && isfinite(jz) && isfinite(phi) &&
                            isfinite(psi);
        if (finite) {
            acc[0] += rho;
            acc[1] += phi;
            acc[2] += psi;
            acc[3] += jx;
            acc[4] += jy;
            acc[5] += jz;
            const double sp = sqrt(jx * jx + jy * jy + jz * jz) / rho;
            acc[6] = fmax(acc[6], sp);
            // interface measure: C_m^2 (1 - C_m)^2 with C1 = (rho + phi - psi)/2, C2 = (rho - phi - psi)/2, C3 = psi
            const double c[3] = {0.5 * (rho + phi - psi), 0.5 * (rho - phi - psi), psi};
#pragma unroll
            for (int m = 0; m < 3; ++m) acc[8 + m] += c[m] * c[m] * (1.0 - c[m]) * (1.0 - c[m]);
        } else {
            acc[7] += 1.0;
        }
    }
#pragma unroll
    for (int s = 0; s < kDiagSlots; ++s) red[s][threadIdx.x] = acc[s];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
#pragma unroll
            for (int s = 0; s < kDiagSlots; ++s) {
                if (s == 6)
                    red[s][threadIdx.x] = fmax(red[s][threadIdx.x], red[s][threadIdx.x + w]);
                else
                    red[s][threadIdx.x] += red[s][threadIdx.x + w];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < kDiagSlots) partial[(int64_t)blockIdx.x * kDiagSlots + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_diag2(const double* __restrict__ partial, int nblocks, double* __restrict__ out)
{
    __shared__ double red[kDiagSlots][256];
    double acc[kDiagSlots] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += 256) {
#pragma unroll
        for (int s = 0; s < kDiagSlots; ++s) {
            const double v = partial[(int64_t)b * kDiagSlots + s];
            acc[s] = (s == 6) ? fmax(acc[s], v) : acc[s] + v;
        }
    }
#pragma unroll
    for (int s = 0; s < kDiagSlots; ++s) red[s][threadIdx.x] = acc[s];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
#pragma unroll
            for (int s = 0; s < kDiagSlots; ++s) {
                if (s == 6)
                    red[s][threadIdx.x] = fmax(red[s][threadIdx.x], red[s][threadIdx.x + w]);
                else
                    red[s][threadIdx.x] += red[s][threadIdx.x + w];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < kDiagSlots) out[threadIdx.x] = red[threadIdx.x][0];
}

template <typename T, typename TIn>
__global__ void k_wet(int n, const TIn* __restrict__ h, double i0, double i1, double i2, T* __restrict__ wet)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= 3 * n) return;
    const int m = j / n;
    const double inv = (m == 0) ? i0 : (m == 1) ? i1 : i2;
    wet[j] = T((double)h[j] * inv);
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

template <typename T, typename TIn>
hipError_t launch_init(const AuxGeom& g, const Phys<acc_t<T>>& P, const TIn* C, const TIn* u, const T* wet, T* state,
                       hipStream_t s)
{
    if (g.lattice == 0)
        hipLaunchKernelGGL((k_init<D2Q9, T, TIn>), grid_for(g.N, 256), dim3(256), 0, s, g, P, C, u, wet, state);
    else
        hipLaunchKernelGGL((k_init<D3Q19, T, TIn>), grid_for(g.N, 256), dim3(256), 0, s, g, P, C, u, wet, state);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fields(const AuxGeom& g, const Phys<acc_t<T>>& P, const T* state, const T* wet, T* F,
                         hipStream_t s)
{
    if (g.lattice == 0) {
        hipLaunchKernelGGL((k_fields1<D2Q9, T>), grid_for(g.N, 256), dim3(256), 0, s, g, state, F);
        hipLaunchKernelGGL((k_fields2<D2Q9, T>), grid_for(g.N, 256), dim3(256), 0, s, g, P, wet, F);
    } else {
        hipLaunchKernelGGL((k_fields1<D3Q19, T>), grid_for(g.N, 256), dim3(256), 0, s, g, state, F);
        hipLaunchKernelGGL((k_fields2<D3Q19, T>), grid_for(g.N, 256), dim3(256), 0, s, g, P, wet, F);
    }
    return hipGetLastError();
}

template <typename T, typename TOut>
hipError_t launch_export_field(const AuxGeom& g, const T* F, int which, TOut* out, hipStream_t s)
{
    // offsets of the stored deviations: C_m, psi: 1/3; rho: 1
    T off = 0;
    if (which <= 2 || which == 5) off = T(1.0 / 3.0);
    if (which == 3) off = T(1);
    hipLaunchKernelGGL((k_export<T, TOut>), grid_for(g.N, 256), dim3(256), 0, s, g.N, F + (int64_t)which * g.N, off,
                       out);
    return hipGetLastError();
}

template <typename T, typename TOut>
hipError_t launch_get_pops(const AuxGeom& g, const T* state, int species, TOut* out, hipStream_t s)
{
    if (g.lattice == 0)
        hipLaunchKernelGGL((k_get_pops<D2Q9, T, TOut>), grid_for(g.N, 256), dim3(256), 0, s, g, state, species, out);
    else
        hipLaunchKernelGGL((k_get_pops<D3Q19, T, TOut>), grid_for(g.N, 256), dim3(256), 0, s, g, state, species, out);
    return hipGetLastError();
}

template <typename T, typename TIn>
hipError_t launch_set_pops(const AuxGeom& g, const TIn* in, int species, T* state, hipStream_t s)
{
    if (g.lattice == 0)
        hipLaunchKernelGGL((k_set_pops<D2Q9, T, TIn>), grid_for(g.N, 256), dim3(256), 0, s, g, in, species, state);
    else
        hipLaunchKernelGGL((k_set_pops<D3Q19, T, TIn>), grid_for(g.N, 256), dim3(256), 0, s, g, in, species, state);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_diag(const AuxGeom& g, const T* state, double* partial, int nblocks, double* out, hipStream_t s)
{
    if (g.lattice == 0)
        hipLaunchKernelGGL((k_diag1<D2Q9, T>), dim3(nblocks), dim3(256), 0, s, g, state, partial);
    else
        hipLaunchKernelGGL((k_diag1<D3Q19, T>), dim3(nblocks), dim3(256), 0, s, g, state, partial);
    hipLaunchKernelGGL(k_diag2, dim3(1), dim3(256), 0, s, partial, nblocks, out);
    return hipGetLastError();
}

template <typename T, typename TIn>
hipError_t launch_wet(int n, const TIn* h, double i0, double i1, double i2, T* wet, hipStream_t s)
{
    hipLaunchKernelGGL((k_wet<T, TIn>), grid_for(3 * (int64_t)n, 256), dim3(256), 0, s, n, h, i0, i1, i2, wet);
    return hipGetLastError();
}

#define TLB_INST_IO(T, TIO)                                                                                   \
    template hipError_t launch_init<T, TIO>(const AuxGeom&, const Phys<acc_t<T>>&, const TIO*, const TIO*,       \
                                            const T*, T*, hipStream_t);                                         \
    template hipError_t launch_export_field<T, TIO>(const AuxGeom&, const T*, int, TIO*, hipStream_t);            \
    template hipError_t launch_get_pops<T, TIO>(const AuxGeom&, const T*, int, TIO*, hipStream_t);                \
    template hipError_t launch_set_pops<T, TIO>(const AuxGeom&, const TIO*, int, T*, hipStream_t);                \
    template hipError_t launch_wet<T, TIO>(int, const TIO*, double, double, double, T*, hipStream_t);

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
