// C ABI of libtlb (declared in include/tlb.h): simulation objects, host and
// device I/O, the step loop and the conservation check.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "../../include/tlb.h"
#include "tlb_internal.hpp"

using namespace tlb;

struct tlb_sim {
    tlb_params p;
    int Q, D;
    int64_t N;
    int dev;
    hipStream_t stream;
    bool own_stream;
    size_t esize;       // bytes per stored value
    void* state[2];     // [nc][Q][N] each
    int cur;            // index of the buffer holding u_t
    void* wet;          // [2][nc][nx*nz] h_m / (alpha^2 kappa_m), or nullptr
    double* hbuf;       // [2][nc][nx*nz] h_m as set (to rescale when kappa changes)
    // adjoint scratch (lazy)
    void* lam[2];
    double* kpart;      // [3][items] kappa-gradient partials
    int64_t kpart_cap;  // items the allocation holds
    tlb_launch adj_launch;
    int cus;            // compute units of the device
    int nc;             // components (3 .. kMaxComp)
    double* dhs;        // [2][3][nx*nz] sink for dL/dh when the caller passes none
    void* seg[2];       // two segment buffers of seg_cap states: one reversed, the next recomputed
    int64_t seg_cap;
    hipStream_t aux;    // recomputes the next segment while the current one is reversed
    hipEvent_t seg_ready[2], main_mark;
    void* fields;       // [11][N] (lazy)
    double* staging;    // device doubles for host I/O (lazy)
    size_t staging_elems;
    double* diag_partial;
    double* diag_out;
    int64_t step;
    bool ready;
    int64_t check_every;
    tlb_launch launch;
    double* hhost;            // [2][nc][nx*nz] h_m as last set from the host (range report)
    int64_t wet_outside[2];   // per wall: values with |4 h_m / (alpha kappa_m)| > 1, -1 if set from device memory
    bool wet_warned;
    int64_t graph_steps;      // steps per captured chain (even), 0: every step launched directly
    hipGraph_t graph;         // the chain from buffer 0, captured on first use
    hipGraphExec_t graph_exec;
};

// Drop the captured chain of steps (its launches hold the parameters and launch shape of capture time).
static void drop_graph(tlb_sim* s)
{
    if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    s->graph_exec = nullptr;
    s->graph = nullptr;
}

static thread_local int g_last_hip = 0;

static tlb_status hip_fail(hipError_t e)
{
    g_last_hip = (int)e;
    return e == hipErrorOutOfMemory ? TLB_ENOMEM : TLB_EHIP;
}

#define HIPCHK(...)                                \
    do {                                           \
        hipError_t e_ = (__VA_ARGS__);             \
        if (e_ != hipSuccess) return hip_fail(e_); \
    } while (0)

extern "C" const char* tlb_status_str(int s)
{
    switch (s) {
        case TLB_OK: return "ok";
        case TLB_EINVAL: return "invalid argument";
        case TLB_ENOMEM: return "out of device memory";
        case TLB_EHIP: return "HIP runtime error";
        case TLB_ENAN: return "non-finite value in the state";
        case TLB_ESTATE: return "call out of order";
        default: return "unknown status";
    }
}

extern "C" int tlb_last_hip_error(void) { return g_last_hip; }
extern "C" int tlb_version(void) { return 500; }

static int ncomp_of(const tlb_params* p) { return p->ncomp == 0 ? 3 : p->ncomp; }

// kappa_m of component m (m < ncomp): kappa[0..2], then kappa_hi.
static double kappa_of(const tlb_params& p, int m) { return m < 3 ? p.kappa[m] : p.kappa_hi[m - 3]; }

static bool params_valid(const tlb_params* p)
{
    if (!p) return false;
    if (p->lattice != TLB_D2Q9 && p->lattice != TLB_D3Q19) return false;
    if (p->prec != TLB_F32 && p->prec != TLB_F64) return false;
    if (p->nx < 3 || p->ny < 3 || p->nz < 1) return false;
    if (p->lattice == TLB_D2Q9 && p->nz != 1) return false;
    if (p->lattice == TLB_D3Q19 && p->nz < 3) return false;
    if (p->walls_y != 0 && p->walls_y != 1) return false;
    for (int m = 0; m < 3; ++m)
        if (!(p->kappa[m] > 0.0) || !isfinite(p->kappa[m])) return false;
    if (!(p->alpha > 0.0) || !isfinite(p->alpha)) return false;
    if (!(p->tau_f > 0.5 && p->tau_g > 0.5 && p->tau_k > 0.5)) return false;
    if (!isfinite(p->tau_f) || !isfinite(p->tau_g) || !isfinite(p->tau_k)) return false;
    if (!isfinite(p->gamma_phi) || !isfinite(p->gamma_psi)) return false;
    if (p->no_advection != 0 && p->no_advection != 1) return false;
    if (p->collision != TLB_BGK && p->collision != TLB_MRT) return false;
    // more than three components (Sec. II.E)
    if (p->ncomp != 0 && (p->ncomp < 3 || p->ncomp > TLB_MAX_COMP)) return false;
    const int nc = ncomp_of(p);
    for (int m = 3; m < nc; ++m)
        if (!(p->kappa_hi[m - 3] > 0.0) || !isfinite(p->kappa_hi[m - 3])) return false;
    if (p->collision == TLB_MRT) {
        if (!(p->tau_bulk > 0.5 && p->tau_ghost > 0.5)) return false;
        if (!isfinite(p->tau_bulk) || !isfinite(p->tau_ghost)) return false;
    }
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    const int Q = p->lattice == TLB_D2Q9 ? 9 : 19;
    const int64_t esize = p->prec == TLB_F32 ? 4 : 8;
    if (p->lattice == TLB_D2Q9) {
        // the D2Q9 step addresses each population array through a descriptor of its own
        if (N * esize > (int64_t)0xFFFFFF00) return false;
    } else {
        // the D3Q19 kernels address each z plane through a descriptor of its own
        if (plane3d_elems(p->nx, p->ny, nc * Q) * esize > (int64_t)0xFFFFFF00) return false;
    }
    return true;
}

template <typename T>
static Phys<T> make_phys(const tlb_params& p)
{
    Phys<T> P;
    const double a2 = p.alpha * p.alpha;
    for (int m = 0; m < kMaxComp; ++m) {
        const double k = m < ncomp_of(&p) ? kappa_of(p, m) : 0.0;
        P.kappa[m] = T(k);
        P.a2kappa[m] = T(a2 * k);
    }
    P.omega[0] = T(1.0 / p.tau_f);
    P.omega[1] = T(1.0 / p.tau_g);
    P.omega[2] = T(1.0 / p.tau_k);
    P.gphi3 = T(3.0 * p.gamma_phi);
    P.gpsi3 = T(3.0 * p.gamma_psi);
    P.adv = p.no_advection ? T(0) : T(1);
    P.mrt_sg = P.mrt_dv = P.mrt_db = T(0);
    if (p.collision == TLB_MRT) {
        P.mrt_sg = T(1.0 / p.tau_ghost);
        P.mrt_dv = T(1.0 / p.tau_f - 1.0 / p.tau_ghost);
        P.mrt_db = T(1.0 / p.tau_bulk - 1.0 / p.tau_ghost);
    }
    return P;
}

static AuxGeom geom(const tlb_sim* s)
{
    AuxGeom g;
    g.lattice = s->p.lattice;
    g.nx = s->p.nx;
    g.ny = s->p.ny;
    g.nz = s->p.nz;
    g.walls = s->p.walls_y;
    g.N = s->N;
    g.nc = s->nc;
    return g;
}

// Reverse sweep: 64-lane strips (58 output columns), four row groups per
// workgroup, the next iteration's pull and lambda rows loaded during the
// current one.  The FP64 transposes hold one wavefront per SIMD, so a
// workgroup fills a compute unit and every item should be resident at once:
// the chunk is sized for one workgroup per compute unit and rounded up so
// that an item takes whole iterations of four rows (chunk + 6 rows in all).
// Measured on MI355X, 512^2 with walls: 22 rows, 216 workgroups, 66 us in
// FP64 against 74 us for single-row groups.
static tlb_launch default_adj_launch(const tlb_params& p, int cus)
{
    tlb_launch l;
    l.width = 64;
    l.height = 4;
    l.variant = 2;
    const int nstrips = (p.nx + 57) / 58;
    // FP32 storage computes in FP32: about 205 registers and 52 KB of LDS, two workgroups per compute unit
    const int per_cu = p.prec == TLB_F32 ? 2 : 1;
    int nch = per_cu * (cus > 0 ? cus : 256) / nstrips;
    if (nch < 1) nch = 1;
    int chunk = (p.ny + nch - 1) / nch;
    chunk += (4 - (chunk + 6) % 4) % 4;
    l.chunk = chunk;
    return l;
}

static void default_launch(tlb_sim* s)
{
    const tlb_params& p = s->p;
    if (p.lattice == TLB_D2Q9) {
        // Measured on MI355X (1024^2): 256-wide strips.  FP64 storage: the
        // prefetch of the next row for three and four components and
        // 16-row items, about 1000 wavefronts in flight, one per SIMD (three
        // components 89.7 against 93.9 us at 8 rows without the prefetch,
        // four 123 against 133 us at 8 rows; five, which spill with the
        // prefetch, 165 against 179 us at 16 rows; 512^2 23.7 against 26.7,
        // 2048^2 353 against 361).  FP32 storage: 8-row items without the
        // prefetch, about 2000 wavefronts in flight (43.0 against 48.5 us).
        // Smaller lattices get shorter chunks rather than fewer workgroups: an item's time is its rows
        // times a row's latency, so a lattice too small to fill the chip runs fastest with one or two
        // rows per item (64^2 FP64: 7.1 us per step at one row against 16.5 at four; 200^2: 9.1
        // against 18.4; 384^2: 19.4 at two against 21.0 at four).
        int w = p.nx >= 256 ? 256 : (p.nx >= 128 ? 128 : 64);
        const int ntx = (p.nx + w - 1) / w;
        const int64_t waves_per_item = w / 64;
        const bool f64 = p.prec == TLB_F64;
        int64_t want_items = (f64 ? 1024 : 2048) / waves_per_item;
        int64_t nch = (want_items + ntx - 1) / ntx;
        int chunk = (int)((p.ny + nch - 1) / nch);
        if (chunk < 1) chunk = 1;
        s->launch.width = w;
        s->launch.height = 1;
        s->launch.chunk = chunk;
        // four components hold one wavefront per SIMD in either storage, where the prefetch of the
        // next row pays; with five it spills
        s->launch.variant = (s->nc == 4 || (f64 && s->nc == 3)) ? 1 : 0;
        s->adj_launch = default_adj_launch(p, s->cus);
    } else {
        // Measured on MI355X (256^3 FP32): 64x4 tiles holding the next plane,
        // ~1000 wavefronts in flight; with FP32 storage the pipelined sweep
        // (loads of plane z+2 in flight during the collision of plane z) is
        // 5% faster.
        // 32 x 8 tiles where 64-wide ones would leave lanes idle (96^3 FP32: 124 us per step against
        // 175); chunks down to one plane for lattices too small to fill the chip (32^3: 12.7 us against
        // 23.7 with four planes).
        const int waste64 = (p.nx + 63) / 64 * 64 - p.nx, waste32 = (p.nx + 31) / 32 * 32 - p.nx;
        int bx = (p.nx >= 64 && waste64 <= waste32) ? 64 : 32, by = bx == 64 ? 4 : 8;
        const int ntx = (p.nx + bx - 1) / bx, nty = (p.ny + by - 1) / by;
        const int64_t waves_per_item = (bx * by) / 64;
        int64_t want_items = 1024 / waves_per_item;
        int64_t nch = (want_items + (int64_t)ntx * nty - 1) / ((int64_t)ntx * nty);
        if (nch < 1) nch = 1;
        int chunk = (int)((p.nz + nch - 1) / nch);
        if (chunk < 1) chunk = 1;
        s->launch.width = bx;
        s->launch.height = by;
        s->launch.chunk = chunk;
        // the pipelined sweep is built for FP32 storage of three or four components (four: 2.11
        // against 2.34 ms with variant 1 at 256^3).  With five FP32 keeps plane z's populations
        // (variant 1: 3.09 against 3.31 ms); in FP64 those would spill, so it pulls plane z twice
        s->launch.variant = p.prec == TLB_F32 ? (s->nc <= 4 ? 2 : 1) : (s->nc > 3 ? 0 : 1);
    }
}

static bool launch_valid(const tlb_sim* s, const tlb_launch* l)
{
    if (l->chunk < 1 || l->variant < 0 || l->variant > 2) return false;
    if (s->p.lattice == TLB_D2Q9)
        return l->variant < 2 && (l->width == 64 || l->width == 128 || l->width == 256);
    // the pipelined sweep is built for FP32 storage of three or four components
    if (l->variant == 2 && (s->p.prec != TLB_F32 || s->nc > 4)) return false;
    const int w = l->width, h = l->height;
    if (w == 32 && h == 8) return true;
    if (w == 64 && h == 4) return true;
    return false;
}

extern "C" tlb_status tlb_create(const tlb_params* params, void* stream, tlb_sim** out)
{
    if (!out || !params_valid(params)) return TLB_EINVAL;
    *out = nullptr;
    tlb_sim* s = new (std::nothrow) tlb_sim();
    if (!s) return TLB_ENOMEM;
    memset(s, 0, sizeof(*s));
    s->p = *params;
    s->Q = params->lattice == TLB_D2Q9 ? 9 : 19;
    s->D = params->lattice == TLB_D2Q9 ? 2 : 3;
    s->N = (int64_t)params->nx * params->ny * params->nz;
    s->esize = params->prec == TLB_F32 ? 4 : 8;
    s->nc = ncomp_of(params);
    hipError_t e = hipGetDevice(&s->dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, s->dev);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e);
    }
    if (stream) {
        s->stream = (hipStream_t)stream;
        s->own_stream = false;
    } else {
        e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete s;
            return hip_fail(e);
        }
        s->own_stream = true;
    }
    const size_t bytes = (size_t)tlb_state_bytes(s);
    for (int b = 0; b < 2; ++b) {
        e = hipMalloc(&s->state[b], bytes);
        // the padding of the D3Q19 blocks is never written by the kernels; zero it once so that raw
        // states compare and checkpoint bit for bit
        if (e == hipSuccess) e = hipMemsetAsync(s->state[b], 0, bytes, s->stream);
        if (e != hipSuccess) {
            tlb_destroy(s);
            return hip_fail(e);
        }
    }
    if (params->walls_y) {
        const size_t nh = (size_t)2 * s->nc * params->nx * params->nz;
        e = hipMalloc(&s->wet, nh * s->esize);
        if (e == hipSuccess) e = hipMemsetAsync(s->wet, 0, nh * s->esize, s->stream);
        if (e == hipSuccess) e = hipMalloc((void**)&s->hbuf, nh * sizeof(double));
        if (e == hipSuccess) e = hipMemsetAsync(s->hbuf, 0, nh * sizeof(double), s->stream);
        if (e != hipSuccess) {
            tlb_destroy(s);
            return hip_fail(e);
        }
    }
    e = hipMalloc((void**)&s->diag_partial, sizeof(double) * kDiagBlocks * kDiagSlots);
    if (e == hipSuccess) e = hipMalloc((void**)&s->diag_out, sizeof(double) * kDiagSlots);
    if (e != hipSuccess) {
        tlb_destroy(s);
        return hip_fail(e);
    }
    default_launch(s);
    *out = s;
    return TLB_OK;
}

extern "C" tlb_status tlb_destroy(tlb_sim* s)
{
    if (!s) return TLB_EINVAL;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    drop_graph(s);
    for (int b = 0; b < 2; ++b)
        if (s->state[b]) (void)hipFree(s->state[b]);
    if (s->wet) (void)hipFree(s->wet);
    if (s->aux) (void)hipStreamSynchronize(s->aux);
    for (void* q : {(void*)s->hbuf, s->lam[0], s->lam[1], (void*)s->kpart, (void*)s->dhs, s->seg[0], s->seg[1]})
        if (q) (void)hipFree(q);
    for (hipEvent_t e : {s->seg_ready[0], s->seg_ready[1], s->main_mark})
        if (e) (void)hipEventDestroy(e);
    if (s->aux) (void)hipStreamDestroy(s->aux);
    if (s->fields) (void)hipFree(s->fields);
    if (s->staging) (void)hipFree(s->staging);
    if (s->diag_partial) (void)hipFree(s->diag_partial);
    if (s->diag_out) (void)hipFree(s->diag_out);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    free(s->hhost);
    delete s;
    return TLB_OK;
}

extern "C" tlb_status tlb_get_params(const tlb_sim* s, tlb_params* out)
{
    if (!s || !out) return TLB_EINVAL;
    *out = s->p;
    return TLB_OK;
}

extern "C" void* tlb_get_stream(const tlb_sim* s) { return s ? (void*)s->stream : nullptr; }

extern "C" tlb_status tlb_get_step(const tlb_sim* s, int64_t* step)
{
    if (!s || !step) return TLB_EINVAL;
    *step = s->step;
    return TLB_OK;
}

extern "C" tlb_status tlb_synchronize(tlb_sim* s)
{
    if (!s) return TLB_EINVAL;
    HIPCHK(hipStreamSynchronize(s->stream));
    return TLB_OK;
}

static tlb_status ensure_staging(tlb_sim* s, size_t elems)
{
    if (s->staging_elems >= elems) return TLB_OK;
    if (s->staging) {
        HIPCHK(hipStreamSynchronize(s->stream));
        HIPCHK(hipFree(s->staging));
        s->staging = nullptr;
        s->staging_elems = 0;
    }
    HIPCHK(hipMalloc((void**)&s->staging, elems * sizeof(double)));
    s->staging_elems = elems;
    return TLB_OK;
}

static tlb_status ensure_fields(tlb_sim* s)
{
    if (s->fields) return TLB_OK;
    HIPCHK(hipMalloc(&s->fields, (size_t)(s->nc + 8) * s->N * s->esize));
    return TLB_OK;
}

// ---------------------------------------------------------------------------
// Wetting parameters
// ---------------------------------------------------------------------------
static tlb_status rescale_wet(tlb_sim* s, int wall)
{
    const int n = s->p.nx * s->p.nz;
    const double a2 = s->p.alpha * s->p.alpha;
    WetScale inv = {};
    for (int m = 0; m < s->nc; ++m) inv.v[m] = 1.0 / (a2 * kappa_of(s->p, m));
    const size_t o = (size_t)wall * s->nc * n;
    const double* h = s->hbuf + o;
    hipError_t e;
    if (s->p.prec == TLB_F32)
        e = launch_wet<float, double>(n, s->nc, h, inv, (float*)s->wet + o, s->stream);
    else
        e = launch_wet<double, double>(n, s->nc, h, inv, (double*)s->wet + o, s->stream);
    HIPCHK(e);
    return TLB_OK;
}

template <typename TIn>
static tlb_status set_wet_impl(tlb_sim* s, int wall, const TIn* h_dev)
{
    const int n = s->p.nx * s->p.nz;
    HIPCHK(launch_convert<TIn, double>(h_dev, s->hbuf + (size_t)wall * s->nc * n, (int64_t)s->nc * n, s->stream));
    return rescale_wet(s, wall);
}

// Wetting parameters outside the range where the wall free energy of Sec. II.B has the closed-form
// wall values (|4 h_m / (alpha kappa_m)| <= 1) are allowed; they are counted, and the first time a
// simulation receives one a warning goes to stderr.
static void count_outside(tlb_sim* s, int wall)
{
    if (!s->hhost) return;
    const int64_t n = (int64_t)s->p.nx * s->p.nz;
    const double* h = s->hhost + (size_t)wall * s->nc * n;
    int64_t c = 0;
    for (int m = 0; m < s->nc; ++m) {
        const double lim = 0.25 * s->p.alpha * kappa_of(s->p, m);
        for (int64_t j = 0; j < n; ++j) c += fabs(h[m * n + j]) > lim;
    }
    s->wet_outside[wall] = c;
    if (c > 0 && !s->wet_warned) {
        s->wet_warned = true;
        fprintf(stderr,
                "libtlb: warning: %lld wetting parameters of wall %d have |4 h_m / (alpha kappa_m)| > 1, outside the "
                "range of the closed-form wall concentrations and contact angles (Sec. II.B); the boundary condition "
                "is still applied as given\n",
                (long long)c, wall);
    }
}

extern "C" tlb_status tlb_wetting_outside_range(const tlb_sim* s, int64_t* count)
{
    if (!s || !count) return TLB_EINVAL;
    if (s->wet_outside[0] < 0 || s->wet_outside[1] < 0) {
        *count = -1;
        return TLB_OK;
    }
    *count = s->wet_outside[0] + s->wet_outside[1];
    return TLB_OK;
}

extern "C" tlb_status tlb_set_wetting(tlb_sim* s, int wall, const double* h)
{
    if (!s || !h || (wall != 0 && wall != 1) || !s->p.walls_y) return TLB_EINVAL;
    const size_t n = (size_t)s->nc * s->p.nx * s->p.nz;
    for (size_t j = 0; j < n; ++j)
        if (!isfinite(h[j])) return TLB_EINVAL;
    if (!s->hhost) {
        s->hhost = (double*)calloc(2 * n, sizeof(double));
        if (!s->hhost) return TLB_ENOMEM;
    }
    memcpy(s->hhost + (size_t)wall * n, h, n * sizeof(double));
    count_outside(s, wall);
    tlb_status st = ensure_staging(s, n);
    if (st) return st;
    HIPCHK(hipMemcpyAsync(s->staging, h, n * sizeof(double), hipMemcpyHostToDevice, s->stream));
    st = set_wet_impl<double>(s, wall, s->staging);
    if (st) return st;
    HIPCHK(hipStreamSynchronize(s->stream));
    return TLB_OK;
}

extern "C" tlb_status tlb_set_wetting_dev(tlb_sim* s, int wall, const void* h_dev)
{
    if (!s || !h_dev || (wall != 0 && wall != 1) || !s->p.walls_y) return TLB_EINVAL;
    s->wet_outside[wall] = -1;  // device values are not inspected on the host
    if (s->p.prec == TLB_F32) return set_wet_impl<float>(s, wall, (const float*)h_dev);
    return set_wet_impl<double>(s, wall, (const double*)h_dev);
}

// ---------------------------------------------------------------------------
// Initialisation
// ---------------------------------------------------------------------------
template <typename T, typename TIn>
static tlb_status init_impl(tlb_sim* s, const TIn* C, const TIn* u)
{
    s->cur = 0;
    HIPCHK(launch_init<T, TIn>(geom(s), make_phys<acc_t<T>>(s->p), C, u, (const T*)s->wet, (T*)s->state[0], s->stream));
    s->step = 0;
    s->ready = true;
    return TLB_OK;
}

extern "C" tlb_status tlb_init_equilibrium(tlb_sim* s, const double* C, const double* u)
{
    if (!s || !C) return TLB_EINVAL;
    const size_t nc = (size_t)s->nc * s->N, nu = u ? (size_t)s->D * s->N : 0;
    tlb_status st = ensure_staging(s, nc + nu);
    if (st) return st;
    HIPCHK(hipMemcpyAsync(s->staging, C, nc * sizeof(double), hipMemcpyHostToDevice, s->stream));
    if (u) HIPCHK(hipMemcpyAsync(s->staging + nc, u, nu * sizeof(double), hipMemcpyHostToDevice, s->stream));
    const double* ud = u ? s->staging + nc : nullptr;
    st = (s->p.prec == TLB_F32) ? init_impl<float, double>(s, s->staging, ud) : init_impl<double, double>(s, s->staging, ud);
    if (st) return st;
    HIPCHK(hipStreamSynchronize(s->stream));
    return TLB_OK;
}

extern "C" tlb_status tlb_init_equilibrium_dev(tlb_sim* s, const void* C, const void* u)
{
    if (!s || !C) return TLB_EINVAL;
    if (s->p.prec == TLB_F32) return init_impl<float, float>(s, (const float*)C, (const float*)u);
    return init_impl<double, double>(s, (const double*)C, (const double*)u);
}

// ---------------------------------------------------------------------------
// Stepping
// ---------------------------------------------------------------------------
template <typename T>
static StepArgs<T> step_args(const tlb_sim* s)
{
    StepArgs<T> a;
    memset(&a, 0, sizeof(a));
    const tlb_params& p = s->p;
    a.wet = (const T*)s->wet;
    a.nx = p.nx;
    a.ny = p.ny;
    a.nz = p.nz;
    a.walls = p.walls_y;
    a.N = s->N;
    a.P = make_phys<acc_t<T>>(p);
    a.Pf = make_phys<float>(p);
    a.chunk = s->launch.chunk;
    if (p.lattice == TLB_D2Q9) {
        a.ntx = (p.nx + s->launch.width - 1) / s->launch.width;
        a.nty = 1;
        a.nchunks = (p.ny + a.chunk - 1) / a.chunk;
    } else {
        a.ntx = (p.nx + s->launch.width - 1) / s->launch.width;
        a.nty = (p.ny + s->launch.height - 1) / s->launch.height;
        a.nchunks = (p.nz + a.chunk - 1) / a.chunk;
    }
    a.nitems = a.ntx * a.nty * a.nchunks;
    return a;
}

template <typename T>
static hipError_t launch_one(const tlb_sim* s, const StepArgs<T>& a)
{
    return (s->p.lattice == TLB_D2Q9)
               ? launch_step2d<T>(a, s->launch.width, s->launch.variant, s->p.collision == TLB_MRT, s->nc,
                                  s->stream)
               : launch_step3d<T>(a, s->launch.width, s->launch.height, s->launch.variant,
                                  s->p.collision == TLB_MRT, s->nc, s->stream);
}

// n steps, each launched directly.
template <typename T>
static tlb_status launch_steps(tlb_sim* s, int64_t n)
{
    StepArgs<T> a = step_args<T>(s);
    for (int64_t t = 0; t < n; ++t) {
        a.src = (const T*)s->state[s->cur];
        a.dst = (T*)s->state[s->cur ^ 1];
        a.flip = s->cur;  // every other step sweeps each chunk the other way
        HIPCHK(launch_one<T>(s, a));
        s->cur ^= 1;
    }
    return TLB_OK;
}

// n steps: whole chains of graph_steps replayed from the captured graph (which starts from buffer 0
// and, being even, ends there), the rest launched directly.
template <typename T>
static tlb_status run_steps(tlb_sim* s, int64_t n)
{
    const int64_t G = s->graph_steps;
    if (G > 0 && n >= G + (s->cur != 0 ? 1 : 0)) {
        if (s->cur != 0) {
            tlb_status st = launch_steps<T>(s, 1);
            if (st) return st;
            --n;
        }
        if (!s->graph_exec) {
            drop_graph(s);  // a graph left by a failed instantiation
            HIPCHK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
            tlb_status st = launch_steps<T>(s, G);  // recorded, not run: cur is back at 0
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(s->stream, &g);
            if (st) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            HIPCHK(e);
            s->graph = g;
            HIPCHK(hipGraphInstantiate(&s->graph_exec, g, nullptr, nullptr, 0));
        }
        for (; n >= G; n -= G) HIPCHK(hipGraphLaunch(s->graph_exec, s->stream));
    }
    return launch_steps<T>(s, n);
}

template <typename T>
static tlb_status step_impl(tlb_sim* s, int64_t nsteps)
{
    while (nsteps > 0) {
        // up to the next conservation check
        int64_t n = nsteps;
        if (s->check_every > 0) n = std::min<int64_t>(n, s->check_every - s->step % s->check_every);
        tlb_status st = run_steps<T>(s, n);
        if (st) return st;
        s->step += n;
        nsteps -= n;
        if (s->check_every > 0 && s->step % s->check_every == 0) {
            tlb_diag d;
            st = tlb_diagnostics(s, &d);
            if (st) return st;
        }
    }
    return TLB_OK;
}

extern "C" tlb_status tlb_set_graph(tlb_sim* s, int64_t steps_per_graph)
{
    if (!s || steps_per_graph < 0 || (steps_per_graph & 1)) return TLB_EINVAL;
    HIPCHK(hipStreamSynchronize(s->stream));
    drop_graph(s);
    s->graph_steps = steps_per_graph;
    return TLB_OK;
}

extern "C" tlb_status tlb_step(tlb_sim* s, int64_t nsteps)
{
    if (!s || nsteps < 0) return TLB_EINVAL;
    if (!s->ready) return TLB_ESTATE;
    return s->p.prec == TLB_F32 ? step_impl<float>(s, nsteps) : step_impl<double>(s, nsteps);
}

template <typename T>
static tlb_status stream_impl(tlb_sim* s, int64_t nsteps)
{
    StepArgs<T> a = step_args<T>(s);
    for (int64_t t = 0; t < nsteps; ++t) {
        a.src = (const T*)s->state[s->cur];
        a.dst = (T*)s->state[s->cur ^ 1];
        a.flip = s->cur;
        HIPCHK(launch_stream_only<T>(a, s->p.lattice, s->launch.width, s->launch.height, s->nc, s->stream));
        s->cur ^= 1;
    }
    return TLB_OK;
}

extern "C" tlb_status tlb_stream_only(tlb_sim* s, int64_t nsteps)
{
    if (!s || nsteps < 0) return TLB_EINVAL;
    if (!s->ready) return TLB_ESTATE;
    return s->p.prec == TLB_F32 ? stream_impl<float>(s, nsteps) : stream_impl<double>(s, nsteps);
}

extern "C" tlb_status tlb_set_check_every(tlb_sim* s, int64_t every)
{
    if (!s || every < 0) return TLB_EINVAL;
    s->check_every = every;
    return TLB_OK;
}

extern "C" tlb_status tlb_set_launch(tlb_sim* s, const tlb_launch* l)
{
    if (!s || !l) return TLB_EINVAL;
    tlb_launch v = *l;
    if (s->p.lattice == TLB_D2Q9) v.height = 1;
    if (v.chunk == 0) {
        tlb_launch d = s->launch;
        default_launch(s);
        v.chunk = s->launch.chunk;
        s->launch = d;
    }
    if (!launch_valid(s, &v)) return TLB_EINVAL;
    if (memcmp(&v, &s->launch, sizeof(v)) != 0) {
        HIPCHK(hipStreamSynchronize(s->stream));
        drop_graph(s);  // the captured launches have the old shape
    }
    s->launch = v;
    return TLB_OK;
}

extern "C" tlb_status tlb_get_launch(const tlb_sim* s, tlb_launch* out)
{
    if (!s || !out) return TLB_EINVAL;
    *out = s->launch;
    return TLB_OK;
}

extern "C" tlb_status tlb_set_adjoint_launch(tlb_sim* s, const tlb_launch* l)
{
    if (!s || !l) return TLB_EINVAL;
    if (s->p.lattice != TLB_D2Q9) return TLB_EINVAL;
    tlb_launch v = *l;
    if (v.height == 0) v.height = 1;
    if (v.chunk == 0) v.chunk = default_adj_launch(s->p, s->cus).chunk;
    if ((v.width != 64 && v.width != 128 && v.width != 256) || v.chunk < 1) return TLB_EINVAL;
    if ((v.height != 1 && v.height != 2 && v.height != 4) || v.width * v.height > 256) return TLB_EINVAL;
    if (v.variant < 0 || v.variant > 2) return TLB_EINVAL;
    s->adj_launch = v;
    return TLB_OK;
}

extern "C" tlb_status tlb_get_adjoint_launch(const tlb_sim* s, tlb_launch* out)
{
    if (!s || !out) return TLB_EINVAL;
    *out = s->adj_launch;
    return TLB_OK;
}

extern "C" tlb_status tlb_device_copy(void* dst, const void* src, int64_t bytes, void* stream)
{
    if (!dst || !src || bytes < 0 || (bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15)) return TLB_EINVAL;
    if (bytes == 0) return TLB_OK;
    HIPCHK(launch_copy16(src, dst, bytes / 16, (hipStream_t)stream));
    return TLB_OK;
}

extern "C" double tlb_bytes_per_node(const tlb_sim* s)
{
    if (!s) return 0.0;
    return 2.0 * s->nc * s->Q * (double)s->esize;
}

// ---------------------------------------------------------------------------
// Readout
// ---------------------------------------------------------------------------
template <typename T, typename TOut>
static tlb_status field_impl(tlb_sim* s, int which, TOut* out)
{
    tlb_status st = ensure_fields(s);
    if (st) return st;
    const AuxGeom g = geom(s);
    HIPCHK(launch_fields<T>(g, make_phys<acc_t<T>>(s->p), (const T*)s->state[s->cur], (const T*)s->wet, (T*)s->fields,
                            s->stream));
    HIPCHK(launch_export_field<T, TOut>(g, (const T*)s->fields, which, out, s->stream));
    return TLB_OK;
}

extern "C" tlb_status tlb_get_field(tlb_sim* s, int which, double* out)
{
    if (!s || !out || field_row(s->nc, which) < 0) return TLB_EINVAL;
    if (!s->ready) return TLB_ESTATE;
    tlb_status st = ensure_staging(s, (size_t)s->N);
    if (st) return st;
    st = (s->p.prec == TLB_F32) ? field_impl<float, double>(s, which, s->staging)
                                : field_impl<double, double>(s, which, s->staging);
    if (st) return st;
    HIPCHK(hipMemcpyAsync(out, s->staging, (size_t)s->N * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return TLB_OK;
}

extern "C" tlb_status tlb_get_field_dev(tlb_sim* s, int which, void* out)
{
    if (!s || !out || field_row(s->nc, which) < 0) return TLB_EINVAL;
    if (!s->ready) return TLB_ESTATE;
    if (s->p.prec == TLB_F32) return field_impl<float, float>(s, which, (float*)out);
    return field_impl<double, double>(s, which, (double*)out);
}

extern "C" tlb_status tlb_get_populations(tlb_sim* s, int species, double* out)
{
    if (!s || !out || species < 0 || species >= s->nc) return TLB_EINVAL;
    if (!s->ready) return TLB_ESTATE;
    const size_t n = (size_t)s->Q * s->N;
    tlb_status st = ensure_staging(s, n);
    if (st) return st;
    const AuxGeom g = geom(s);
    hipError_t e = (s->p.prec == TLB_F32)
                       ? launch_get_pops<float, double>(g, (const float*)s->state[s->cur], species, s->staging, s->stream)
                       : launch_get_pops<double, double>(g, (const double*)s->state[s->cur], species, s->staging,
                                                         s->stream);
    HIPCHK(e);
    HIPCHK(hipMemcpyAsync(out, s->staging, n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return TLB_OK;
}

extern "C" tlb_status tlb_get_populations_dev(tlb_sim* s, int species, void* out)
{
    if (!s || !out || species < 0 || species >= s->nc) return TLB_EINVAL;
    if (!s->ready) return TLB_ESTATE;
    const AuxGeom g = geom(s);
    hipError_t e = (s->p.prec == TLB_F32)
                       ? launch_get_pops<float, float>(g, (const float*)s->state[s->cur], species, (float*)out, s->stream)
                       : launch_get_pops<double, double>(g, (const double*)s->state[s->cur], species, (double*)out,
                                                         s->stream);
    HIPCHK(e);
    return TLB_OK;
}

extern "C" tlb_status tlb_set_populations(tlb_sim* s, int species, const double* in)
{
    if (!s || !in || species < 0 || species >= s->nc) return TLB_EINVAL;
    const size_t n = (size_t)s->Q * s->N;
    tlb_status st = ensure_staging(s, n);
    if (st) return st;
    HIPCHK(hipMemcpyAsync(s->staging, in, n * sizeof(double), hipMemcpyHostToDevice, s->stream));
    const AuxGeom g = geom(s);
    hipError_t e = (s->p.prec == TLB_F32)
                       ? launch_set_pops<float, double>(g, s->staging, species, (float*)s->state[s->cur], s->stream)
                       : launch_set_pops<double, double>(g, s->staging, species, (double*)s->state[s->cur], s->stream);
    HIPCHK(e);
    HIPCHK(hipStreamSynchronize(s->stream));
    s->ready = true;
    return TLB_OK;
}

extern "C" tlb_status tlb_set_populations_dev(tlb_sim* s, int species, const void* in)
{
    if (!s || !in || species < 0 || species >= s->nc) return TLB_EINVAL;
    const AuxGeom g = geom(s);
    hipError_t e = (s->p.prec == TLB_F32)
                       ? launch_set_pops<float, float>(g, (const float*)in, species, (float*)s->state[s->cur], s->stream)
                       : launch_set_pops<double, double>(g, (const double*)in, species, (double*)s->state[s->cur],
                                                         s->stream);
    HIPCHK(e);
    s->ready = true;
    return TLB_OK;
}

extern "C" tlb_status tlb_diagnostics(tlb_sim* s, tlb_diag* out)
{
    if (!s || !out) return TLB_EINVAL;
    if (!s->ready) return TLB_ESTATE;
    const AuxGeom g = geom(s);
    hipError_t e = (s->p.prec == TLB_F32)
                       ? launch_diag<float>(g, (const float*)s->state[s->cur], s->diag_partial, kDiagBlocks,
                                            s->diag_out, s->stream)
                       : launch_diag<double>(g, (const double*)s->state[s->cur], s->diag_partial, kDiagBlocks,
                                             s->diag_out, s->stream);
    HIPCHK(e);
    double h[kDiagSlots];
    HIPCHK(hipMemcpyAsync(h, s->diag_out, sizeof(h), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (int m = 0; m < 3; ++m) {
        out->mass[m] = h[m];
        out->momentum[m] = h[3 + m];
        out->interface[m] = h[8 + m];
    }
    for (int l = 0; l < TLB_MAX_COMP - 3; ++l) {
        const bool on = l < s->nc - 3;
        out->mass_hi[l] = on ? h[11 + l] : 0.0;
        out->interface_hi[l] = on ? h[11 + (s->nc - 3) + l] : 0.0;
    }
    out->max_speed = h[6];
    out->nonfinite = (int64_t)h[7];
    out->step = s->step;
    return out->nonfinite ? TLB_ENAN : TLB_OK;
}

// ---------------------------------------------------------------------------
// Raw checkpoints
// ---------------------------------------------------------------------------
extern "C" int64_t tlb_state_bytes(const tlb_sim* s)
{
    if (!s) return 0;
    if (s->p.lattice == TLB_D3Q19)
        return (int64_t)s->p.nz * plane3d_elems(s->p.nx, s->p.ny, s->nc * s->Q) * (int64_t)s->esize;
    return (int64_t)s->nc * s->Q * s->N * (int64_t)s->esize;
}

extern "C" tlb_status tlb_save_state(tlb_sim* s, void* dst, int64_t* step)
{
    if (!s || !dst) return TLB_EINVAL;
    if (!s->ready) return TLB_ESTATE;
    HIPCHK(hipMemcpyAsync(dst, s->state[s->cur], (size_t)tlb_state_bytes(s), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (step) *step = s->step;
    return TLB_OK;
}

extern "C" tlb_status tlb_load_state(tlb_sim* s, const void* src, int64_t step)
{
    if (!s || !src || step < 0) return TLB_EINVAL;
    HIPCHK(hipMemcpyAsync(s->state[s->cur], src, (size_t)tlb_state_bytes(s), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->step = step;
    s->ready = true;
    return TLB_OK;
}

extern "C" tlb_status tlb_save_state_dev(tlb_sim* s, void* dst)
{
    if (!s || !dst) return TLB_EINVAL;
    if (!s->ready) return TLB_ESTATE;
    HIPCHK(hipMemcpyAsync(dst, s->state[s->cur], (size_t)tlb_state_bytes(s), hipMemcpyDeviceToDevice, s->stream));
    return TLB_OK;
}

extern "C" tlb_status tlb_load_state_dev(tlb_sim* s, const void* src, int64_t step)
{
    if (!s || !src || step < 0) return TLB_EINVAL;
    HIPCHK(hipMemcpyAsync(s->state[s->cur], src, (size_t)tlb_state_bytes(s), hipMemcpyDeviceToDevice, s->stream));
    s->step = step;
    s->ready = true;
    return TLB_OK;
}

// ---------------------------------------------------------------------------
// Parameters that may change between runs, and the adjoint
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Contact angles <-> wetting parameters (Sec. II.B, II.D), host only.
// ---------------------------------------------------------------------------
// Phi(h) = kappa (s+^3 - s-^3), s+- = sqrt(1 +- 4h/(alpha kappa)): the solid tension difference
// gamma_sn - gamma_sm equals alpha (Phi_m - Phi_n) / 12; Phi is increasing on |h| <= alpha kappa / 4.
static double wet_phi(double k, double a, double h)
{
    const double r = 4.0 * h / (a * k);
    const double sp = sqrt(fmax(0.0, 1.0 + r)), sm = sqrt(fmax(0.0, 1.0 - r));
    return k * (sp * sp * sp - sm * sm * sm);
}

static bool wet_params_ok(const double* kappa, double alpha)
{
    if (!kappa || !(alpha > 0.0) || !isfinite(alpha)) return false;
    for (int m = 0; m < 3; ++m)
        if (!(kappa[m] > 0.0) || !isfinite(kappa[m])) return false;
    return true;
}

// h with Phi(h) = phi by bisection on [-alpha kappa/4, alpha kappa/4]; false if out of range.
static bool wet_h_of_phi(double k, double a, double phi, double* h)
{
    double lo = -0.25 * a * k, hi = 0.25 * a * k;
    if (phi < wet_phi(k, a, lo) || phi > wet_phi(k, a, hi)) return false;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (wet_phi(k, a, mid) < phi)
            lo = mid;
        else
            hi = mid;
    }
    *h = 0.5 * (lo + hi);
    return true;
}

extern "C" tlb_status tlb_contact_angles(const double* kappa, double alpha, const double* h, double* theta_out)
{
    if (!wet_params_ok(kappa, alpha) || !h || !theta_out) return TLB_EINVAL;
    double phi[3];
    for (int m = 0; m < 3; ++m) {
        if (!isfinite(h[m]) || fabs(4.0 * h[m] / (alpha * kappa[m])) > 1.0) return TLB_EINVAL;
        phi[m] = wet_phi(kappa[m], alpha, h[m]);
    }
    const double rad = 180.0 / 3.14159265358979323846;
    for (int j = 0; j < 3; ++j) {
        const int m = j, n = (j + 1) % 3;
        double c = (phi[m] - phi[n]) / (2.0 * (kappa[m] + kappa[n]));
        c = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
        theta_out[j] = acos(c) * rad;
    }
    return TLB_OK;
}

extern "C" tlb_status tlb_wetting_from_angles(const double* kappa, double alpha, double theta12, double theta23,
                                              double* h_out)
{
    if (!wet_params_ok(kappa, alpha) || !h_out || !isfinite(theta12) || !isfinite(theta23)) return TLB_EINVAL;
    if (theta12 < 0.0 || theta12 > 180.0 || theta23 < 0.0 || theta23 > 180.0) return TLB_EINVAL;
    const double deg = 3.14159265358979323846 / 180.0;
    // Phi_1 - Phi_2 and Phi_2 - Phi_3 are fixed by the angles; Phi_3 = t is the remaining freedom,
    // chosen so that sum_m h_m / kappa_m = 0 (which increases with t).
    const double d12 = 2.0 * (kappa[0] + kappa[1]) * cos(theta12 * deg);
    const double d23 = 2.0 * (kappa[1] + kappa[2]) * cos(theta23 * deg);
    const double off[3] = {d12 + d23, d23, 0.0};
    double lo = -1e300, hi = 1e300;
    for (int m = 0; m < 3; ++m) {  // t range on which every Phi_m stays attainable
        const double pmin = wet_phi(kappa[m], alpha, -0.25 * alpha * kappa[m]);
        const double pmax = wet_phi(kappa[m], alpha, 0.25 * alpha * kappa[m]);
        lo = fmax(lo, pmin - off[m]);
        hi = fmin(hi, pmax - off[m]);
    }
    if (!(lo <= hi)) return TLB_EINVAL;
    auto redundancy = [&](double t, double* h) {
        double g = 0.0;
        for (int m = 0; m < 3; ++m) {
            if (!wet_h_of_phi(kappa[m], alpha, t + off[m], &h[m])) h[m] = (t + off[m] > 0 ? 0.25 : -0.25) * alpha * kappa[m];
            g += h[m] / kappa[m];
        }
        return g;
    };
    double h[3];
    if (redundancy(lo, h) > 0.0 || redundancy(hi, h) < 0.0) return TLB_EINVAL;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (redundancy(mid, h) < 0.0)
            lo = mid;
        else
            hi = mid;
    }
    redundancy(0.5 * (lo + hi), h);
    for (int m = 0; m < 3; ++m) h_out[m] = h[m];
    return TLB_OK;
}

extern "C" tlb_status tlb_set_kappa(tlb_sim* s, const double* kappa)
{
    if (!s || !kappa) return TLB_EINVAL;
    for (int m = 0; m < s->nc; ++m)
        if (!(kappa[m] > 0.0) || !isfinite(kappa[m])) return TLB_EINVAL;
    HIPCHK(hipStreamSynchronize(s->stream));
    drop_graph(s);  // the captured launches hold the old coefficients
    for (int m = 0; m < s->nc; ++m) (m < 3 ? s->p.kappa[m] : s->p.kappa_hi[m - 3]) = kappa[m];
    if (s->p.walls_y) {
        tlb_status st = rescale_wet(s, 0);
        if (!st) st = rescale_wet(s, 1);
        if (st) return st;
        for (int w = 0; w < 2; ++w)
            if (s->wet_outside[w] >= 0) count_outside(s, w);
    }
    return TLB_OK;
}

// Work decomposition of the reverse sweep: strips of (width - 6) output columns times chunks of rows.
static void adj_items(const tlb_sim* s, int& nstrips, int& nchunks)
{
    const int O = s->adj_launch.width - 6;
    nstrips = (s->p.nx + O - 1) / O;
    nchunks = (s->p.ny + s->adj_launch.chunk - 1) / s->adj_launch.chunk;
}

static int64_t adj_nitems(const tlb_sim* s)
{
    int a, b;
    adj_items(s, a, b);
    return (int64_t)a * b;
}

static tlb_status adj_alloc(tlb_sim* s, int64_t seg_states)
{
    const size_t sb = (size_t)tlb_state_bytes(s);
    for (int b = 0; b < 2; ++b)
        if (!s->lam[b]) HIPCHK(hipMalloc(&s->lam[b], sb));
    const int64_t items = adj_nitems(s);
    if (items > s->kpart_cap) {
        if (s->kpart) {
            HIPCHK(hipStreamSynchronize(s->stream));
            HIPCHK(hipFree(s->kpart));
            s->kpart = nullptr;
            s->kpart_cap = 0;
        }
        HIPCHK(hipMalloc((void**)&s->kpart, (size_t)3 * items * sizeof(double)));
        s->kpart_cap = items;
    }
    if (!s->dhs) HIPCHK(hipMalloc((void**)&s->dhs, (size_t)6 * s->p.nx * s->p.nz * sizeof(double)));
    if (seg_states > s->seg_cap) {
        HIPCHK(hipStreamSynchronize(s->stream));
        if (s->aux) HIPCHK(hipStreamSynchronize(s->aux));
        for (int b = 0; b < 2; ++b)
            if (s->seg[b]) {
                HIPCHK(hipFree(s->seg[b]));
                s->seg[b] = nullptr;
            }
        s->seg_cap = 0;
        for (int b = 0; b < 2; ++b) HIPCHK(hipMalloc(&s->seg[b], sb * (size_t)seg_states));
        s->seg_cap = seg_states;
    }
    if (seg_states > 0 && !s->aux) {
        for (int b = 0; b < 2; ++b) HIPCHK(hipEventCreateWithFlags(&s->seg_ready[b], hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&s->main_mark, hipEventDisableTiming));
        HIPCHK(hipStreamCreateWithFlags(&s->aux, hipStreamNonBlocking));
    }
    return TLB_OK;
}

// One reverse step.  kassign: write the kappa partials of this step (a single step, or the first of a
// pass) instead of adding to them, so that they need no clearing.
template <typename T>
static tlb_status adj_step(tlb_sim* s, const void* u, const void* lam1, void* lam0, double* dh, double* kpart,
                           bool kassign)
{
    AdjArgs<T> a;
    memset(&a, 0, sizeof(a));
    a.u = (const T*)u;
    a.lam1 = (const T*)lam1;
    a.lam0 = (T*)lam0;
    a.wet = (const T*)s->wet;
    a.dh = dh;
    a.kpart = kpart;
    a.kassign = kassign ? 1 : 0;
    a.nx = s->p.nx;
    a.ny = s->p.ny;
    a.walls = s->p.walls_y;
    a.N = s->N;
    a.chunk = s->adj_launch.chunk;
    adj_items(s, a.nstrips, a.nchunks);
    a.nitems = a.nstrips * a.nchunks;
    a.P = make_phys<acc_t<T>>(s->p);
    a.Pf = make_phys<float>(s->p);
    HIPCHK(launch_adjoint_sweep<T>(a, s->adj_launch.width, s->adj_launch.height, s->adj_launch.variant, s->stream));
    return TLB_OK;
}

static tlb_status adj_step_any(tlb_sim* s, const void* u, const void* lam1, void* lam0, double* dh, bool kassign,
                               double* kpart = nullptr)
{
    if (!kpart) kpart = s->kpart;
    return s->p.prec == TLB_F32 ? adj_step<float>(s, u, lam1, lam0, dh, kpart, kassign)
                                : adj_step<double>(s, u, lam1, lam0, dh, kpart, kassign);
}

// Reduce the kappa partials into dkappa (+=) after a reverse step or pass.
static tlb_status kpart_reduce(tlb_sim* s, double* dkappa)
{
    if (dkappa) HIPCHK(launch_reduce_items(s->kpart, adj_nitems(s), dkappa, s->stream));
    return TLB_OK;
}

// The reverse sweep addresses a whole state through one buffer descriptor (32-bit byte offsets).
static bool adj_fits(const tlb_sim* s) { return tlb_state_bytes(s) <= (int64_t)0xFFFFFF00; }

// dh accumulation target [2][3][nx]: the caller's array, or a scratch sink.
static double* dh_target(tlb_sim* s, double* dh) { return dh ? dh : s->dhs; }

extern "C" tlb_status tlb_adjoint_seed_dev(tlb_sim* s, const void* dLdC, void* lam)
{
    if (!s || !lam) return TLB_EINVAL;
    if (s->p.lattice != TLB_D2Q9 || s->p.collision != TLB_BGK || s->nc != 3 || !adj_fits(s)) return TLB_EINVAL;
    const AuxGeom g = geom(s);
    hipError_t e = (s->p.prec == TLB_F32) ? launch_adjoint_seed<float>(g, (const float*)dLdC, (float*)lam, s->stream)
                                          : launch_adjoint_seed<double>(g, (const double*)dLdC, (double*)lam, s->stream);
    HIPCHK(e);
    return TLB_OK;
}

extern "C" tlb_status tlb_adjoint_step_dev(tlb_sim* s, const void* state, const void* lam_in, void* lam_out,
                                           double* dh, double* dkappa)
{
    if (!s || !state || !lam_in || !lam_out || lam_in == lam_out) return TLB_EINVAL;
    if (s->p.lattice != TLB_D2Q9 || s->p.collision != TLB_BGK || s->nc != 3 || !adj_fits(s)) return TLB_EINVAL;
    tlb_status st = adj_alloc(s, 0);
    if (!st) st = adj_step_any(s, state, lam_in, lam_out, dh_target(s, dh), true);
    if (!st) st = kpart_reduce(s, dkappa);
    return st;
}

extern "C" tlb_status tlb_adjoint_step(tlb_sim* s, const void* state, void* lam, double* dh, double* dkappa)
{
    if (!s || !state || !lam) return TLB_EINVAL;
    if (s->p.lattice != TLB_D2Q9 || s->p.collision != TLB_BGK || s->nc != 3 || !adj_fits(s)) return TLB_EINVAL;
    tlb_status st = adj_alloc(s, 0);
    if (!st) st = adj_step_any(s, state, lam, s->lam[0], dh_target(s, dh), true);
    if (!st) st = kpart_reduce(s, dkappa);
    if (st) return st;
    HIPCHK(hipMemcpyAsync(lam, s->lam[0], (size_t)tlb_state_bytes(s), hipMemcpyDeviceToDevice, s->stream));
    return TLB_OK;
}

// ---------------------------------------------------------------------------
// Reverse step without allocation.  Its scratch (the per-item kappa partials,
// their reduction partials and, when the caller passes no dh array, a sink
// for dL/dh) lives in one file-scope device array per GPU, so the call needs
// no hipMalloc; every call on a GPU shares that GPU's copy.
// ---------------------------------------------------------------------------
constexpr int64_t kScratchDoubles = TLB_NOALLOC_SCRATCH_BYTES / 8;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each GPU (null until looked up)

// Device address of this GPU's copy of `scratch`, looked up once per device with that device current.
static tlb_status scratch_of(int dev, double** out)
{
    if (dev < 0 || dev >= kMaxDevices) return TLB_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        HIPCHK(hipGetDevice(&cur));
        if (cur != dev) HIPCHK(hipSetDevice(dev));
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess && e2 != hipSuccess) return hip_fail(e2);
        }
        if (e != hipSuccess) return hip_fail(e);
        if (!ptr) return TLB_EHIP;
        g_scratch_ptr[dev] = (double*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return TLB_OK;
}

extern "C" int64_t tlb_adjoint_step_noalloc_scratch(const tlb_sim* s)
{
    if (!s) return 0;
    return (3 * adj_nitems(s) + 6 * (int64_t)s->p.nx * s->p.nz) * (int64_t)sizeof(double);
}

extern "C" tlb_status tlb_adjoint_step_noalloc(tlb_sim* s, const void* state, const void* lam_in, void* lam_out,
                                               double* dh, double* dkappa)
{
    if (!s || !state || !lam_in || !lam_out || lam_in == lam_out) return TLB_EINVAL;
    if (s->p.lattice != TLB_D2Q9 || s->p.collision != TLB_BGK || s->nc != 3 || !adj_fits(s)) return TLB_EINVAL;
    if (tlb_adjoint_step_noalloc_scratch(s) > TLB_NOALLOC_SCRATCH_BYTES) return TLB_EINVAL;
    double* base = nullptr;
    tlb_status st = scratch_of(s->dev, &base);
    if (st) return st;
    const int64_t items = adj_nitems(s);
    double* kpart = base;             // [3][items], written by the step (whatever the last call left)
    double* sink = base + 3 * items;  // [2][3][nx*nz] when dh is NULL
    if (!dh) {
        HIPCHK(launch_fill0(sink, 6 * (int64_t)s->p.nx * s->p.nz, s->stream));
        dh = sink;
    }
    st = adj_step_any(s, state, lam_in, lam_out, dh, true, kpart);
    if (st) return st;
    if (dkappa) HIPCHK(launch_reduce_items(kpart, items, dkappa, s->stream));
    return TLB_OK;
}

extern "C" int64_t tlb_checkpoint_slots(int64_t nsteps, int64_t every)
{
    if (nsteps < 1 || every < 1) return 0;
    return (nsteps + every - 1) / every;
}

extern "C" tlb_status tlb_forward_checkpointed(tlb_sim* s, int64_t nsteps, int64_t every, void* ckpt)
{
    if (!s || !ckpt || nsteps < 1 || every < 1) return TLB_EINVAL;
    if (!s->ready) return TLB_ESTATE;
    const size_t sb = (size_t)tlb_state_bytes(s);
    for (int64_t t = 0; t < nsteps; t += every) {
        HIPCHK(hipMemcpyAsync((char*)ckpt + sb * (size_t)(t / every), s->state[s->cur], sb, hipMemcpyDeviceToDevice,
                              s->stream));
        const int64_t n = (t + every <= nsteps) ? every : nsteps - t;
        tlb_status st = tlb_step(s, n);
        if (st) return st;
    }
    return TLB_OK;
}

template <typename T>
static tlb_status recompute(tlb_sim* s, const void* from, int64_t count, void* seg, hipStream_t stream)
{
    // seg[0] = from; seg[k] = step(seg[k-1]) for k < count
    const size_t sb = (size_t)tlb_state_bytes(s);
    HIPCHK(hipMemcpyAsync(seg, from, sb, hipMemcpyDeviceToDevice, stream));
    StepArgs<T> a = step_args<T>(s);
    for (int64_t k = 1; k < count; ++k) {
        a.src = (const T*)((const char*)seg + sb * (size_t)(k - 1));
        a.dst = (T*)((char*)seg + sb * (size_t)k);
        a.flip = (int)(k & 1);
        HIPCHK((s->p.lattice == TLB_D2Q9)
                   ? launch_step2d<T>(a, s->launch.width, s->launch.variant, s->p.collision == TLB_MRT, s->nc, stream)
                   : launch_step3d<T>(a, s->launch.width, s->launch.height, s->launch.variant,
                                      s->p.collision == TLB_MRT, s->nc, stream));
    }
    return TLB_OK;
}

static tlb_status recompute_any(tlb_sim* s, const void* from, int64_t count, void* seg, hipStream_t stream)
{
    return s->p.prec == TLB_F32 ? recompute<float>(s, from, count, seg, stream)
                                : recompute<double>(s, from, count, seg, stream);
}

extern "C" tlb_status tlb_adjoint_backward(tlb_sim* s, int64_t nsteps, int64_t every, const void* ckpt,
                                           const void* dLdC, double* dh, double* dkappa)
{
    if (!s || !ckpt || nsteps < 1 || every < 1) return TLB_EINVAL;
    if (s->p.lattice != TLB_D2Q9 || s->p.collision != TLB_BGK || s->nc != 3 || !adj_fits(s)) return TLB_EINVAL;
    tlb_status st = adj_alloc(s, every);
    if (st) return st;
    const size_t sb = (size_t)tlb_state_bytes(s);
    st = tlb_adjoint_seed_dev(s, dLdC, s->lam[0]);
    if (st) return st;
    int cur = 0;
    bool first = true;  // the first reverse step writes the kappa partials, the others add to them
    const int64_t nseg = tlb_checkpoint_slots(nsteps, every);
    auto seg_t0 = [&](int64_t seg) { return seg * every; };
    auto seg_len = [&](int64_t seg) { return ((seg_t0(seg) + every <= nsteps) ? every : nsteps - seg_t0(seg)); };
    auto seg_from = [&](int64_t seg) { return (const void*)((const char*)ckpt + sb * (size_t)seg); };
    // Segments are reversed from the last to the first, in two buffers that take turns: while the
    // reverse steps of segment `seg` run on the simulation's stream from one buffer, the forward
    // recompute of segment seg - 1 runs on the auxiliary stream into the other one.  The auxiliary
    // stream starts each recompute after all work queued on the simulation's stream so far (which
    // includes the reverse steps that last read that buffer, and the caller's checkpoints), and the
    // reverse steps of a segment start after its recompute.
    st = recompute_any(s, seg_from(nseg - 1), seg_len(nseg - 1), s->seg[0], s->stream);
    if (st) return st;
    for (int64_t i = 0; i < nseg; ++i) {
        const int64_t seg = nseg - 1 - i;
        const int b = (int)(i & 1);
        if (seg > 0) {
            HIPCHK(hipEventRecord(s->main_mark, s->stream));
            HIPCHK(hipStreamWaitEvent(s->aux, s->main_mark, 0));
            st = recompute_any(s, seg_from(seg - 1), seg_len(seg - 1), s->seg[b ^ 1], s->aux);
            if (st) return st;
            HIPCHK(hipEventRecord(s->seg_ready[b ^ 1], s->aux));
        }
        if (i > 0) HIPCHK(hipStreamWaitEvent(s->stream, s->seg_ready[b], 0));
        const int64_t t0 = seg_t0(seg), t1 = t0 + seg_len(seg);
        for (int64_t t = t1 - 1; t >= t0; --t) {
            const void* u = (const char*)s->seg[b] + sb * (size_t)(t - t0);
            st = adj_step_any(s, u, s->lam[cur], s->lam[cur ^ 1], dh_target(s, dh), first);
            if (st) return st;
            first = false;
            cur ^= 1;
        }
    }
    return kpart_reduce(s, dkappa);
}
