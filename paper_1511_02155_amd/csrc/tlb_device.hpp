// Device-side building blocks of the ternary free-energy LB step for gfx950:
// lattice tables, the storage shift, and the per-node thermodynamics,
// equilibria and BGK collision (Sec. III and IV of arXiv:1511.02155).
//
// Storage shift.  Populations are kept in HBM as deviations from a constant,
// direction-symmetric reference r_{s,i}: f: w_i (the rest equilibrium at
// rho = 1, v = 0); g: 0; each k: psi_ref at i = 0, 0 otherwise (psi_ref =
// 1/NC for NC components, the state with every C_m = 1/NC).
//
// Components (Sec. II.E): NC = 3 is the ternary model; for NC > 3 the
// variables are rho = sum_m C_m, phi = C1 - C2 and psi_l = C_l (l >= 3), with
// one k population set per psi_l stored after f and g.
// Propagation and half-way bounce-back map a uniform, direction-symmetric
// field onto itself, and collision is affine, so the deviations obey the same
// update; keeping O(1) constants out of the stored values keeps FP32 rounding
// at the scale of the deviations.  Every moment and equilibrium below is
// written directly in terms of the deviations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tlb {

constexpr double kPsiRef = 1.0 / 3.0;  // psi_ref of the ternary model
constexpr int kMaxComp = 5;            // largest number of components the kernels are built for

template <int NC>
__host__ __device__ constexpr double psi_ref()
{
    return 1.0 / NC;
}

// ---------------------------------------------------------------------------
// Lattices (velocity order documented in include/tlb.h).
// ---------------------------------------------------------------------------
struct D2Q9 {
    static constexpr int Q = 9;
    static constexpr int D = 2;
    static constexpr int ex[9] = {0, 1, -1, 0, 0, 1, 1, -1, -1};
    static constexpr int ey[9] = {0, 0, 0, 1, -1, 1, -1, 1, -1};
    static constexpr int ez[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int opp[9] = {0, 2, 1, 4, 3, 8, 7, 6, 5};
};

struct D3Q19 {
    static constexpr int Q = 19;
    static constexpr int D = 3;
    static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, 1, -1, -1};
    static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 1, 1, -1, -1, 0, 0, 0, 0};
    static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
    static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
};

template <class L>
__host__ __device__ constexpr int e2(int i)
{
    return L::ex[i] * L::ex[i] + L::ey[i] * L::ey[i] + L::ez[i] * L::ez[i];
}

// Lattice weights: D2Q9 4/9, 1/9, 1/36; D3Q19 1/3, 1/18, 1/36 (Sec. IV).
template <class L>
__host__ __device__ constexpr double weight(int i)
{
    return L::D == 2 ? (e2<L>(i) == 0 ? 4.0 / 9.0 : e2<L>(i) == 1 ? 1.0 / 9.0 : 1.0 / 36.0)
                     : (e2<L>(i) == 0 ? 1.0 / 3.0 : e2<L>(i) == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

template <class L>
__host__ __device__ constexpr int ecomp(int i, int a)
{
    return a == 0 ? L::ex[i] : a == 1 ? L::ey[i] : L::ez[i];
}

// Gradient weights w_i^{aa} (assigned by velocity class: D3Q19 values of
// Sec. IV; D2Q9 values 1/9, -1/18, -1/72 satisfying the same second-moment
// conditions) and w_i^{ab} = e_a e_b / 12 on diagonals.
template <class L>
__host__ __device__ constexpr double wdiag(int i, int a)
{
    return e2<L>(i) == 0 ? 0.0
           : e2<L>(i) == 1
               ? (ecomp<L>(i, a) != 0 ? (L::D == 2 ? 1.0 / 9.0 : 5.0 / 36.0)
                                      : (L::D == 2 ? -1.0 / 18.0 : -1.0 / 9.0))
               : (ecomp<L>(i, a) != 0 ? -1.0 / 72.0 : 1.0 / 36.0);
}

template <class L>
__host__ __device__ constexpr double woff(int i, int a, int b)
{
    return e2<L>(i) == 2 ? ecomp<L>(i, a) * ecomp<L>(i, b) / 12.0 : 0.0;
}

// Moments of the multiple-relaxation-time collision of f that relax at a rate
// of their own (the others all share the ghost rate): the energy moment
// (D2Q9 3|e|^2 - 4, D3Q19 19|e|^2 - 30; bulk viscosity) and the viscous stress
// moments, a basis of the traceless second moments (D2Q9 e_x^2 - e_y^2,
// e_x e_y; D3Q19 3e_x^2 - |e|^2, e_y^2 - e_z^2, e_x e_y, e_y e_z, e_x e_z).
// In an orthogonal moment basis containing them, the collision is
//   f* = f - s_g d - (s_v - s_g) P_stress d - (s_b - s_g) P_energy d,
// d = f - f^eq, with P the orthogonal projections onto their spans.
template <class L>
__host__ __device__ constexpr double mrt_energy(int i)
{
    return L::D == 2 ? 3.0 * e2<L>(i) - 4.0 : 19.0 * e2<L>(i) - 30.0;
}
template <class L>
__host__ __device__ constexpr int mrt_nstress()
{
    return L::D == 2 ? 2 : 5;
}
template <class L>
__host__ __device__ constexpr double mrt_stress(int k, int i)
{
    const int x = L::ex[i], y = L::ey[i], z = L::ez[i];
    if (L::D == 2) return k == 0 ? x * x - y * y : x * y;
    return k == 0 ? 3 * x * x - e2<L>(i) : k == 1 ? y * y - z * z : k == 2 ? x * y : k == 3 ? y * z : x * z;
}
template <class L>
__host__ __device__ constexpr double mrt_energy_norm()
{
    double s = 0.0;
    for (int i = 0; i < L::Q; ++i) s += mrt_energy<L>(i) * mrt_energy<L>(i);
    return s;
}
template <class L>
__host__ __device__ constexpr double mrt_stress_norm(int k)
{
    double s = 0.0;
    for (int i = 0; i < L::Q; ++i) s += mrt_stress<L>(k, i) * mrt_stress<L>(k, i);
    return s;
}

// Storage reference r_{s,i} (see the header comment).
template <class L, int NC = 3>
__host__ __device__ constexpr double ref(int s, int i)
{
    return s == 0 ? weight<L>(i) : (s >= 2 && i == 0 ? psi_ref<NC>() : 0.0);
}

// ---------------------------------------------------------------------------
// D3Q19 state layout: plane-major blocks.  The nodes of one z plane are
// numbered m = x + nx*y and grouped into blocks of 64 consecutive m; a block
// stores the NQ = NC*Q populations of its nodes population-major ([NQ][64]),
// the blocks of a plane follow one another (the last one padded), and so do
// the planes.  A wavefront pulling one row of a tile then reads a few
// contiguous runs of NQ*64 values instead of NQ separate arrays (on MI355X
// the 256^3 FP32 step went from 1.85 to 1.62 ms; runs of one species per
// plane instead of all NQ populations per block measured 1.66 ms), and each
// plane is addressed through a buffer descriptor of its own, so byte offsets
// stay below 2^32 for any nz.  (D2Q9 states are species-major [NC][Q][N].)
// ---------------------------------------------------------------------------
constexpr int kBlock3d = 64;
__host__ __device__ constexpr int64_t plane3d_elems(int nx, int ny, int nq)
{
    return ((int64_t)nx * ny + kBlock3d - 1) / kBlock3d * nq * kBlock3d;
}
// Element of population j (= s*Q + i) of in-plane node m within its plane.
__host__ __device__ constexpr int64_t plane3d_index(int64_t m, int nq, int j)
{
    return ((m / kBlock3d) * nq + j) * kBlock3d + (m % kBlock3d);
}

// ---------------------------------------------------------------------------
// Raw buffer access.  A buffer resource covers one species array; loads and
// stores take a per-lane 32-bit byte offset (voffset) and a wavefront-uniform
// byte offset (soffset), so the address arithmetic of the lattice pull runs
// on the scalar unit.  The third resource word is the raw (untyped) access
// configuration of gfx9-family targets.
// ---------------------------------------------------------------------------
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ Rsrc make_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRsrcWord3);
}

template <typename T>
__device__ __forceinline__ T bload(Rsrc r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ float bload<float>(Rsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ double bload<double>(Rsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}

// Stores take a cache-policy operand: 0 is the default; kStoreStream sets the
// non-temporal bit (gfx950: "nt"), which writes the line toward memory without
// keeping it in the caches.  That pays where the stored state is far larger
// than the 256 MB Infinity Cache, so that the next step cannot find it there
// anyway, and costs where the state fits (the next step then reads it from
// memory instead of the cache).
constexpr int kStoreStream = 2;
// A state buffer beyond this size is stored with kStoreStream by the kernels that opt in.
constexpr int64_t kStreamStoreBytes = (int64_t)256 << 20;

template <typename T, int POL = 0>
__device__ __forceinline__ void bstore(T v, Rsrc r, uint32_t voff, uint32_t soff)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "FP32 or FP64 values");
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, POL);
    } else {
        typedef uint32_t u2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, (int)voff, (int)soff, POL);
    }
}

// ---------------------------------------------------------------------------
// Parameters in the form the kernels use.
// ---------------------------------------------------------------------------
template <typename T>
struct Phys {
    T kappa[kMaxComp];
    T a2kappa[kMaxComp];  // alpha^2 kappa_m
    T omega[3];    // 1/tau for f, g, k
    T gphi3, gpsi3;  // Gamma_phi / c_s^2, Gamma_psi / c_s^2
    T adv;           // 1: g^eq, k^eq carry the velocity terms; 0: diffusive Cahn-Hilliard
    // multiple relaxation times of f: the ghost rate s_g = 1/tau_ghost and the differences
    // s_v - s_g (stress moments, s_v = 1/tau_f) and s_b - s_g (energy moment, s_b = 1/tau_bulk)
    T mrt_sg, mrt_dv, mrt_db;
};

// Arithmetic type of the per-node computations for a storage type T.  Both
// storage precisions compute in FP64: populations are converted on load and
// rounded once on store, so FP32 storage adds one rounding per value and
// step and nothing else (the rounding of FP32 arithmetic in the moments,
// stencils and equilibria would otherwise dominate the FP32 error).
template <typename T>
struct Acc {
    using type = double;
};
template <typename T>
using acc_t = typename Acc<T>::type;

// Moments of one node from its (shifted) populations.
template <typename T, int NC = 3>
struct Moments {
    T drho;   // rho - 1
    T jx, jy, jz;
    T phi;
    T dpsi;   // psi_3 - psi_ref
    T dpsx[NC > 3 ? NC - 3 : 1];  // psi_l - psi_ref for l = 4 .. NC
};

// k points to the NC - 2 k population sets, Q values apart.  C: arithmetic type of the sums.
template <typename C, class L, int NC = 3, typename T>
__device__ __forceinline__ Moments<C, NC> moments_as(const T* f, const T* g, const T* k)
{
    Moments<C, NC> m;
    C r = 0, jx = 0, jy = 0, jz = 0, ph = 0, ps[NC - 2];
#pragma unroll
    for (int l = 0; l < NC - 2; ++l) ps[l] = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const C fi = C(f[i]);
        r += fi;
        if (L::ex[i] == 1) jx += fi;
        if (L::ex[i] == -1) jx -= fi;
        if (L::ey[i] == 1) jy += fi;
        if (L::ey[i] == -1) jy -= fi;
        if (L::ez[i] == 1) jz += fi;
        if (L::ez[i] == -1) jz -= fi;
        ph += C(g[i]);
#pragma unroll
        for (int l = 0; l < NC - 2; ++l) ps[l] += C(k[l * L::Q + i]);
    }
    m.drho = r;
    m.jx = jx;
    m.jy = jy;
    m.jz = jz;
    m.phi = ph;
    m.dpsi = ps[0];
#pragma unroll
    for (int l = 1; l < NC - 2; ++l) m.dpsx[l - 1] = ps[l];
    return m;
}

template <class L, int NC = 3, typename T>
__device__ __forceinline__ Moments<acc_t<T>, NC> moments(const T* f, const T* g, const T* k)
{
    return moments_as<acc_t<T>, L, NC>(f, g, k);
}

// Concentration deviations dC_m = C_m - 1/NC from the moments:
// C1 = (rho + phi - sum psi)/2, C2 = (rho - phi - sum psi)/2, C_l = psi_l
// (Sec. II.C, II.E), with rho = 1 + drho and psi_l = 1/NC + dpsi_l.
template <typename T, int NC = 3>
__device__ __forceinline__ void conc_dev(const Moments<T, NC>& m, T dc[NC])
{
    T sp = m.dpsi;
#pragma unroll
    for (int l = 0; l < NC - 3; ++l) sp += m.dpsx[l];
    dc[0] = T(0.5) * (m.drho + m.phi - sp);
    dc[1] = T(0.5) * (m.drho - m.phi - sp);
    dc[2] = m.dpsi;
#pragma unroll
    for (int l = 0; l < NC - 3; ++l) dc[3 + l] = m.dpsx[l];
}

// Chemical potentials mu_phi, mu_psi (of psi_3) of Sec. III from dC_m and lap C_m.
template <typename T, int NC = 3>
__device__ __forceinline__ void chem_potentials(const Phys<T>& P, const T dc[NC], const T lC[NC], T& mu_phi,
                                                T& mu_psi)
{
    T mu[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const T c = T(psi_ref<NC>()) + dc[m];
        mu[m] = P.kappa[m] * c * (T(1) - c) * (T(1) - T(2) * c) - P.a2kappa[m] * lC[m];
    }
    mu_phi = T(0.5) * (mu[0] - mu[1]);
    mu_psi = mu[2] - T(0.5) * (mu[0] + mu[1]);
}

// Per-node collision.  Inputs: the node's shifted populations f, g, k (in
// place -> post-collision), its moments, the concentration deviations dC,
// their gradients gC[m][a] and Laplacians lC[m].
//   mu_m   = kappa_m C_m (1 - C_m)(1 - 2 C_m) - alpha^2 kappa_m lap C_m
//   mu_phi = (mu_1 - mu_2)/2,  mu_psi = mu_3 - (mu_1 + mu_2)/2          (Sec. III)
//   p_b    = rho/3 + sum_m kappa_m/2 C_m^2 (1 - C_m)(1 - 3 C_m)        (Sec. III)
//   Lambda = alpha^2 sum_m kappa_m C_m lap C_m
//   T_ab   = alpha^2 sum_m kappa_m d_a C_m d_b C_m
//   f_i^eq = w_i [ (p_b - Lambda)/c_s^2 + rho U_i ] + (1/c_s^2) sum_ab w_i^{ab} T_ab
//   g_i^eq = w_i [ Gamma_phi mu_phi / c_s^2 + phi U_i ],  k_i^eq likewise (eq. eqdistfbinary)
//   U_i    = e_i.v / c_s^2 + (e_i.v)^2 / (2 c_s^4) - v^2 / (2 c_s^2)
//   rest populations from the mass constraints; BGK with 1/tau per species.
//
// collide_core reads the pre-collision populations through ld(s, i) and hands each post-collision
// value to st(s, i, v) (species s: 0 f, 1 g, 2 + l the k set of psi_{3+l}; v in the arithmetic
// type, rounded to the storage type by the caller); every value is read and written once, in the
// same order for every caller, except that MRT reads f_i a second time.
template <class L, bool MRT = false, int NC = 3, typename T, typename Ld, typename St>
__device__ __forceinline__ void collide_core(const Phys<T>& P, const Moments<T, NC>& mo, const T dc[NC],
                                             const T gC[NC][3], const T lC[NC], Ld ld, St st)
{
    // T: arithmetic type.  MRT: f relaxes with multiple relaxation times (g and k always with BGK).
    // k_l relaxes with the k rate and mu_psi_l = mu_l - (mu_1 + mu_2)/2 (Sec. II.E).
    const T third = T(1.0 / 3.0);
    const T cref = T(psi_ref<NC>());
    T mu[NC];
    T pbx = mo.drho * third;  // p_b - 1/3 (the 1/3 is the reference pressure of the shifted f)
    T lam = 0;
    T Txx = 0, Tyy = 0, Tzz = 0, Txy = 0, Tyz = 0, Tzx = 0;
#pragma unroll
    for (int m = 0; m < NC; ++m) {
        const T c = cref + dc[m];
        const T omc = T(1) - c;
        mu[m] = P.kappa[m] * c * omc * (T(1) - T(2) * c) - P.a2kappa[m] * lC[m];
        pbx += T(0.5) * P.kappa[m] * c * c * omc * (T(1) - T(3) * c);
        lam += P.a2kappa[m] * c * lC[m];
        const T gx = gC[m][0], gy = gC[m][1], gz = gC[m][2];
        Txx += P.a2kappa[m] * gx * gx;
        Tyy += P.a2kappa[m] * gy * gy;
        Txy += P.a2kappa[m] * gx * gy;
        if (L::D == 3) {
            Tzz += P.a2kappa[m] * gz * gz;
            Tyz += P.a2kappa[m] * gy * gz;
            Tzx += P.a2kappa[m] * gz * gx;
        }
    }
    const T mu_phi = T(0.5) * (mu[0] - mu[1]);
    constexpr int NK = NC - 2;
    T Bk[NK], psi[NK];
#pragma unroll
    for (int l = 0; l < NK; ++l) {
        Bk[l] = P.gpsi3 * (mu[2 + l] - T(0.5) * (mu[0] + mu[1]));
        psi[l] = cref + (l == 0 ? mo.dpsi : mo.dpsx[l > 0 ? l - 1 : 0]);
    }

    const T rho = T(1) + mo.drho;
    const T irho = T(1) / rho;
    const T vx = mo.jx * irho, vy = mo.jy * irho, vz = (L::D == 3) ? mo.jz * irho : T(0);
    const T vv = vx * vx + vy * vy + vz * vz;

    const T A = T(3) * (pbx - lam);
    const T Bp = P.gphi3 * mu_phi;
    const T wf = P.omega[0], wg = P.omega[1], wk = P.omega[2];

    // i > 0: equilibrium and relaxation in place; the rest population last,
    // from the mass constraints.
    T sf = 0, sg = 0, sk[NK];
#pragma unroll
    for (int l = 0; l < NK; ++l) sk[l] = 0;
    constexpr int NS = mrt_nstress<L>();
    T dq[MRT ? L::Q : 1];         // MRT: f_i - f_i^eq
    T me = 0, ms[MRT ? NS : 1];   // MRT: energy and stress moments of f - f^eq
    if constexpr (MRT) {
#pragma unroll
        for (int q = 0; q < NS; ++q) ms[q] = 0;
    }
    // Directions come in pairs e_j = -e_i with the same weights (w_i and the second-order w_i^ab are
    // even in e), so an equilibrium splits into a part even in e, shared by the pair, and an odd part
    // of opposite signs: U_i = Ue + Uo, U_j = Ue - Uo with Uo = 3 e_i.v, Ue = 9/2 (e_i.v)^2 - 3/2 v^2.
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const int j = L::opp[i];
        if (j < i) continue;  // each pair once, from its lower index
        const T w = T(weight<L>(i));
        const T ev = T(L::ex[i]) * vx + T(L::ey[i]) * vy + T(L::ez[i]) * vz;
        const T Ue = T(4.5) * ev * ev - T(1.5) * vv, Uo = T(3) * ev;
        T G = T(3 * wdiag<L>(i, 0)) * Txx + T(3 * wdiag<L>(i, 1)) * Tyy +
              T(3 * woff<L>(i, 0, 1)) * Txy;
        if (L::D == 3)
            G += T(3 * wdiag<L>(i, 2)) * Tzz + T(3 * woff<L>(i, 1, 2)) * Tyz +
                 T(3 * woff<L>(i, 2, 0)) * Tzx;
        const T fe = w * (A + rho * Ue) + G, fo = w * rho * Uo;
        // velocity terms of g^eq, k^eq (absent without advection)
        const T Uae = P.adv * Ue, Uao = P.adv * Uo;
        const T ge = w * (Bp + mo.phi * Uae), go = w * mo.phi * Uao;
        T ke[NK], ko[NK];
#pragma unroll
        for (int l = 0; l < NK; ++l) {
            ke[l] = w * (Bk[l] + psi[l] * Uae);
            ko[l] = w * psi[l] * Uao;
        }
        sf += T(2) * fe;
        sg += T(2) * ge;
#pragma unroll
        for (int l = 0; l < NK; ++l) sk[l] += T(2) * ke[l];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int d = h == 0 ? i : j;
            const T sgn = h == 0 ? T(1) : T(-1);
            const T feq = fe + sgn * fo, geq = ge + sgn * go;
            const T fi = ld(0, d), gi = ld(1, d);
            T ki[NK];
#pragma unroll
            for (int l = 0; l < NK; ++l) ki[l] = ld(2 + l, d);
            if constexpr (MRT) {
                dq[d] = fi - feq;
            } else {
                st(0, d, fi + wf * (feq - fi));
            }
            st(1, d, gi + wg * (geq - gi));
#pragma unroll
            for (int l = 0; l < NK; ++l) st(2 + l, d, ki[l] + wk * ((ke[l] + sgn * ko[l]) - ki[l]));
        }
        if constexpr (MRT) {
            // the energy and stress coefficients are even in e: the pair enters its moments as a sum
            const T ds = dq[i] + dq[j];
            me += T(mrt_energy<L>(i)) * ds;
#pragma unroll
            for (int q = 0; q < NS; ++q)
                if (mrt_stress<L>(q, i) != 0.0) ms[q] += T(mrt_stress<L>(q, i)) * ds;
        }
    }
    const T f0 = ld(0, 0), g0 = ld(1, 0);
    if constexpr (MRT) {
        // the rest population has no stress moment; it enters the energy moment
        dq[0] = f0 - (mo.drho - sf);
        me += T(mrt_energy<L>(0)) * dq[0];
        me *= P.mrt_db * T(1.0 / mrt_energy_norm<L>());
#pragma unroll
        for (int q = 0; q < NS; ++q) ms[q] *= P.mrt_dv * T(1.0 / mrt_stress_norm<L>(q));
        st(0, 0, f0 - P.mrt_sg * dq[0] - T(mrt_energy<L>(0)) * me);
        // the projections back onto a pair share their even coefficients
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            const int j = L::opp[i];
            if (j < i) continue;
            T c = T(mrt_energy<L>(i)) * me;
#pragma unroll
            for (int q = 0; q < NS; ++q)
                if (mrt_stress<L>(q, i) != 0.0) c += T(mrt_stress<L>(q, i)) * ms[q];
            st(0, i, ld(0, i) - P.mrt_sg * dq[i] - c);
            st(0, j, ld(0, j) - P.mrt_sg * dq[j] - c);
        }
    } else {
        st(0, 0, f0 + wf * ((mo.drho - sf) - f0));
    }
    st(1, 0, g0 + wg * ((mo.phi - sg) - g0));
#pragma unroll
    for (int l = 0; l < NK; ++l) {
        const T k0 = ld(2 + l, 0);
        const T dps = l == 0 ? mo.dpsi : mo.dpsx[l > 0 ? l - 1 : 0];
        st(2 + l, 0, k0 + wk * ((dps - sk[l]) - k0));
    }
}

// collide_core on arrays, in place: f, g and the NC - 2 k sets (Q values apart) in storage type S,
// each rounded once on the update.
template <class L, bool MRT = false, int NC = 3, typename T, typename S>
__device__ __forceinline__ void collide(const Phys<T>& P, const Moments<T, NC>& mo, const T dc[NC],
                                        const T gC[NC][3], const T lC[NC], S* f, S* g, S* k)
{
    auto ld = [&](int s, int i) -> T { return T(s == 0 ? f[i] : s == 1 ? g[i] : k[(s - 2) * L::Q + i]); };
    auto st = [&](int s, int i, T v) {
        if (s == 0)
            f[i] = S(v);
        else if (s == 1)
            g[i] = S(v);
        else
            k[(s - 2) * L::Q + i] = S(v);
    };
    collide_core<L, MRT, NC>(P, mo, dc, gC, lC, ld, st);
}

// Equilibrium populations (shifted) of given fields; used by initialisation.
template <class L, int NC = 3, typename T, typename S>
__device__ __forceinline__ void equilibrium(const Phys<T>& P, const Moments<T, NC>& mo, const T dc[NC],
                                            const T gC[NC][3], const T lC[NC], S* f, S* g, S* k)
{
    Phys<T> Q = P;
    Q.omega[0] = Q.omega[1] = Q.omega[2] = T(1);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) f[i] = g[i] = S(0);
#pragma unroll
    for (int i = 0; i < (NC - 2) * L::Q; ++i) k[i] = S(0);
    collide<L, false, NC>(Q, mo, dc, gC, lC, f, g, k);
}

}  // namespace tlb
