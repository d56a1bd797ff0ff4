// Batched D2Q9 ternary LB: many independent lattices of uneven size and
// parameters advanced together.
//
// One time step of the whole batch is one persistent launch per stream group
// (the domains split into up to four groups of nearly equal work, each on its
// own stream, so that one group's launch fills the compute units another's
// leaves idle as it drains): a grid sized to
// the number of workgroups the GPU holds at once, whose workgroups take
// (domain, strip, chunk) work items from eight queues (one per XCD, filled
// largest domain first and balanced by load) and steal from the other queues
// once their own is empty.  The kernel boundary is the per-step barrier; the
// queue counters of the next step are cleared inside the kernel, so a chain
// of steps can be captured once in a hipGraph and replayed.  Each work item
// runs the same strip sweep as the single-lattice kernel, or (variant 2, for
// domains with nx + 3 <= workgroup width) a flat sweep over the domain's
// padded rows laid end to end, with the same arithmetic, so a domain's result
// is bit-for-bit the one a single tlb_sim of that domain produces.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/tlb.h"
#include "tlb_sweep2d.hpp"

namespace tlb {

template <typename T>
struct DomDesc {
    int64_t off;      // element offset of the domain's state in a state buffer
    int64_t wet_off;  // element offset of its wetting array, or -1 (no walls)
    int32_t nx, ny, walls, chunk, ntx, nchunks;
    int32_t flat;  // 0: strip sweep (chunk = rows per item); 1: flat sweep (chunk = segments per item)
    Phys<acc_t<T>> P;
};

template <typename T>
struct BatchArgs {
    const T* src;
    T* dst;
    const T* wet;
    const DomDesc<T>* doms;
    const int2* items;  // {domain, strip << 16 | chunk}
    const int* qstart;  // [9]: queue k holds items [qstart[k], qstart[k+1])
    // (flat items: {domain, first segment | count << 16 | downward << 31})
    int* counters;      // [2][8]
    int parity;
};

constexpr int kQueues = 8;
constexpr int kMaxGroups = 4;  // stream groups a batch's domains can be split over

// Pull of node (x, y) addressed per lane: the loads of pull2d (same sources,
// same half-way bounce-back) with the row folded into the lane's offset.  The
// byte offsets of the three source rows and columns are formed once; a
// direction adds one of each and its own array offset.
template <typename T>
__device__ __forceinline__ void pull_flat(Rsrc src, uint32_t N, int nx, int ny, bool walls, int x, int y, T* p)
{
    constexpr uint32_t ES = sizeof(T);
    const uint32_t cx[3] = {(uint32_t)x * ES, (uint32_t)(x == 0 ? nx - 1 : x - 1) * ES,
                            (uint32_t)(x == nx - 1 ? 0 : x + 1) * ES};  // columns x, x-1, x+1
    const uint32_t r0 = (uint32_t)y * (uint32_t)nx * ES;
    const uint32_t ry[3] = {r0, y == 0 ? (uint32_t)(ny - 1) * (uint32_t)nx * ES : r0 - (uint32_t)nx * ES,
                            y == ny - 1 ? 0u : r0 + (uint32_t)nx * ES};  // rows y, y-1, y+1
    const bool blo = walls && y == 0, bhi = walls && y == ny - 1;
    const uint32_t own = r0 + cx[0];
    const uint32_t NB = N * ES;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int ex = L9::ex[i], ey = L9::ey[i];
        const bool bb = (ey == 1) ? blo : (ey == -1) ? bhi : false;
        const uint32_t from = ry[ey == 0 ? 0 : (ey == 1 ? 1 : 2)] + cx[ex == 0 ? 0 : (ex == 1 ? 1 : 2)];
        const uint32_t vo = bb ? own + (uint32_t)L9::opp[i] * NB : from + (uint32_t)i * NB;
#pragma unroll
        for (int s = 0; s < 3; ++s) p[9 * s + i] = bload<T>(src, vo, (uint32_t)(9 * s) * NB);
    }
}

template <typename T, int W>
struct FlatLds {
    acc_t<T> c[3][4 * W];  // C_m of virtual position v at [m][v mod 4W]
};

template <typename T, int W, bool FLAT>
struct BatchLds {
    Sweep2Lds<T, W> strip;
};
template <typename T, int W>
struct BatchLds<T, W, true> {
    union {
        Sweep2Lds<T, W> strip;
        FlatLds<T, W> flat;
    };
};

// Flat sweep of one work item of a domain with nx + 3 <= W: segments
// [seg0, seg1), downwards if `down`.  A strip of W
// lanes would leave W - nx lanes of every row idle; here the rows, each padded
// with its two periodic halo columns (P = nx + 2 positions: the copy of
// column nx-1, columns 0 .. nx-1, the copy of column 0), are laid end to end
// and lane t of segment s owns position v = s W + t.  The x neighbours of an
// interior position are v -+ 1 and the rows below and above are v -+ P, so a
// node's nine neighbours lie within the segments before and after its own.
// Consecutive items of a domain alternate between upward and downward sweeps
// (neighbouring items meet at shared segments, as the strips do).  The item
// runs in the strip sweep's pipeline: C_m of segment k+1 (pulled and
// summed by every lane, halo lanes included) goes to a ring of four segments
// in LDS and its populations stay in registers; one barrier; then the
// interior nodes of segment k take their stencils from the ring and collide.
// Positions beyond the ends are periodic images (y periodic) or never read
// (walls: ghost rows are made from the node's own row).  Every value is formed
// by the same operations in the same order as in the strip sweep (pull,
// moments, concentrations, ghost rows, stencil9, collide), so the results are
// bitwise those of the strip sweep.
template <typename T, int W>
__device__ __forceinline__ void flat2d(const StepArgs<T>& A, int seg0, int seg1, bool down, FlatLds<T, W>& S)
{
    using C = acc_t<T>;
    constexpr int RM = 4 * W - 1;
    auto& ring = S.c;
    const int t = threadIdx.x;
    const int nx = A.nx, ny = A.ny, P = nx + 2, NP = ny * P;
    const bool walls = A.walls != 0;
    const uint32_t NU = (uint32_t)A.N;
    const uint32_t sbytes = (uint32_t)(27 * A.N * (int64_t)sizeof(T));
    const Rsrc rs = make_rsrc(A.src, sbytes);
    const Rsrc rd = make_rsrc(A.dst, sbytes);

    // physical column of padded position xp
    auto col_of = [&](int xp) { return xp == 0 ? nx - 1 : (xp == P - 1 ? 0 : xp - 1); };

    // Segment s: every lane pulls its position's node into p, its moments
    // into mo and C_m into the ring.
    auto cpass = [&](int s, T* p, Moments<C, 3>& mo) {
        const int v = s * W + t;
        int u = v;
        bool ok = v >= 0 && v < NP;
        if (!walls) {
            u = v % NP;
            u = u < 0 ? u + NP : u;
            ok = true;
        }
        if (ok) {
            const int y = (int)((uint32_t)u / (uint32_t)P);
            const int x = col_of(u - y * P);
            pull_flat<T>(rs, NU, nx, ny, walls, x, y, p);
            mo = moments<L9, 3>(p, p + 9, p + 18);
            C c[3];
            conc_dev<C, 3>(mo, c);
#pragma unroll
            for (int m = 0; m < 3; ++m) ring[m][v & RM] = c[m];
        }
    };
    // Segment s: stencils, collision and store of its interior nodes.
    auto bpass = [&](int s, T* p, const Moments<C, 3>& mo) {
        const int v = s * W + t;
        const int y = (int)((uint32_t)v / (uint32_t)P), xp = v - y * P;
        if (v < NP && xp >= 1 && xp <= nx) {
            const int x = xp - 1;
            const int xl = col_of(xp - 1), xr = col_of(xp + 1);
            const bool glo = walls && y == 0, ghi = walls && y == ny - 1;
            C gC[3][3], lC[3], dc[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const C bl = ring[m][(v - 1) & RM], bc = ring[m][v & RM], br = ring[m][(v + 1) & RM];
                C al = ring[m][(v - P - 1) & RM], ac = ring[m][(v - P) & RM], ar = ring[m][(v - P + 1) & RM];
                C cl = ring[m][(v + P - 1) & RM], cc = ring[m][(v + P) & RM], cr = ring[m][(v + P + 1) & RM];
                // ghost rows (reading R8): C_m(ghost) = C_m(adjacent fluid node) + h_m / (alpha^2 kappa_m)
                if (glo) {
                    const T* __restrict__ wt = A.wet + m * nx;
                    al = bl + C(wt[xl]);
                    ac = bc + C(wt[x]);
                    ar = br + C(wt[xr]);
                }
                if (ghi) {
                    const T* __restrict__ wt = A.wet + (3 + m) * nx;
                    cl = bl + C(wt[xl]);
                    cc = bc + C(wt[x]);
                    cr = br + C(wt[xr]);
                }
                stencil9<C>(ac, al + ar, ar - al, bc, bl + br, br - bl, cc, cl + cr, cr - cl, 1, gC[m], lC[m]);
                dc[m] = bc;
            }
            collide<L9, false, 3>(A.P, mo, dc, gC, lC, p, p + 9, p + 18);
            const uint32_t vo = (uint32_t)(y * nx + x) * (uint32_t)sizeof(T);
#pragma unroll
            for (int q = 0; q < 27; ++q) bstore<T>(p[q], rd, vo, (uint32_t)q * NU * (uint32_t)sizeof(T));
        }
    };

    // Two population buffers take turns; one barrier per segment (the ring
    // slot written next is none of the three a lane may still be reading).
    T P0[27], P1[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) P0[i] = P1[i] = T(0);
    Moments<C, 3> M0, M1;
    const int d = down ? -1 : 1;
    const int kb = d > 0 ? seg0 : seg1 - 1;  // first segment collided
    const int n = seg1 - seg0;
    cpass(kb - d, P1, M1);
    cpass(kb, P0, M0);
    int j = 0;
    for (; j + 1 < n; j += 2) {
        const int k = kb + j * d;
        cpass(k + d, P1, M1);
        __syncthreads();
        bpass(k, P0, M0);
        cpass(k + 2 * d, P0, M0);
        __syncthreads();
        bpass(k + d, P1, M1);
    }
    if (j < n) {
        const int k = kb + j * d;
        cpass(k + d, P1, M1);
        __syncthreads();
        bpass(k, P0, M0);
    }
}

// MODE 0: strip sweep; 1: strip sweep with a one-row prefetch; 2: flat sweep
// for domains with nx + 3 <= W (flat in the descriptor), strips for the rest.
template <typename T, int W, int MODE>
__global__ __launch_bounds__(W) __attribute__((amdgpu_waves_per_eu(step2d_waves<T, MODE == 1 ? 1 : 0>())))
void k_batch2d(BatchArgs<T> B)
{
    constexpr int DEPTH = MODE == 1 ? 1 : 0;
    __shared__ BatchLds<T, W, MODE == 2> S;
    __shared__ int s_item;
    if (blockIdx.x == 0 && threadIdx.x < kQueues) B.counters[(B.parity ^ 1) * kQueues + threadIdx.x] = 0;
    // Workgroups are dispatched round-robin over the XCDs: start on the
    // queue of this workgroup's XCD, then move on to the others.
    int q = blockIdx.x & (kQueues - 1);
    int empty = 0;
    while (empty < kQueues) {
        if (threadIdx.x == 0) {
            const int k = atomicAdd(&B.counters[B.parity * kQueues + q], 1);
            const int idx = B.qstart[q] + k;
            s_item = (idx < B.qstart[q + 1]) ? idx : -1;
        }
        __syncthreads();
        // the item is the same for the whole workgroup: keep it (and the domain's parameters) in
        // scalar registers
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (it < 0) {
            q = (q + 1) & (kQueues - 1);
            ++empty;
            continue;
        }
        const int2 w = B.items[it];
        const DomDesc<T>& D = B.doms[w.x];
        StepArgs<T> A;
        A.src = B.src + D.off;
        A.dst = B.dst + D.off;
        A.wet = D.wet_off >= 0 ? B.wet + D.wet_off : nullptr;
        A.nx = D.nx;
        A.ny = D.ny;
        A.nz = 1;
        A.walls = D.walls;
        A.N = (int64_t)D.nx * D.ny;
        A.chunk = D.chunk;
        A.nchunks = D.nchunks;
        A.ntx = D.ntx;
        A.nty = 1;
        A.nitems = D.ntx * D.nchunks;
        A.flip = B.parity;  // every other step sweeps each item the other way
        A.P = D.P;
        if constexpr (MODE == 2) {
            if (D.flat)
                flat2d<T, W>(A, w.y & 0xffff, (w.y & 0xffff) + ((w.y >> 16) & 0x7fff), (w.y < 0) != (B.parity != 0),
                             S.flat);
            else
                sweep2d<T, W, DEPTH>(A, w.y >> 16, w.y & 0xffff, S.strip);
        } else {
            sweep2d<T, W, DEPTH>(A, w.y >> 16, w.y & 0xffff, S.strip);
        }
        __syncthreads();
    }
}

template <typename T>
static hipError_t launch_batch2d(const BatchArgs<T>& a, int width, int depth, int grid, hipStream_t s)
{
#define TLB_LB(WW, DD)                                                                         \
    if (width == WW && depth == DD) {                                                          \
        hipLaunchKernelGGL((k_batch2d<T, WW, DD>), dim3(grid), dim3(WW), 0, s, a);             \
        return hipGetLastError();                                                              \
    }
    TLB_LB(64, 0)
    TLB_LB(128, 0)
    TLB_LB(256, 0)
    TLB_LB(64, 1)
    TLB_LB(128, 1)
    TLB_LB(256, 1)
    TLB_LB(64, 2)
    TLB_LB(128, 2)
    TLB_LB(256, 2)
#undef TLB_LB
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t occupancy_batch2d(int width, int depth, int* blocks_per_cu)
{
#define TLB_OB(WW, DD)                                                                                 \
    if (width == WW && depth == DD)                                                                    \
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch2d<T, WW, DD>, WW, 0);
    TLB_OB(64, 0)
    TLB_OB(128, 0)
    TLB_OB(256, 0)
    TLB_OB(64, 1)
    TLB_OB(128, 1)
    TLB_OB(256, 1)
    TLB_OB(64, 2)
    TLB_OB(128, 2)
    TLB_OB(256, 2)
#undef TLB_OB
    return hipErrorInvalidValue;
}

}  // namespace tlb

using namespace tlb;

struct tlb_batch {
    int ndom;
    int prec;
    size_t esize;
    std::vector<tlb_params> p;
    std::vector<int64_t> off;      // state offsets (elements)
    std::vector<int64_t> wet_off;  // wetting offsets (elements) or -1
    int64_t state_elems, wet_elems, total_nodes, max_nodes;
    hipStream_t stream;
    bool own_stream;
    void* state[2];
    int cur;  // buffer holding u_t; also the queue-counter parity of the next step
    void* wet;
    void* doms;  // DomDesc<T>[ndom]
    int2* items;
    int* qstart;    // [kMaxGroups][kQueues + 1]
    int* counters;  // [kMaxGroups][2][kQueues]
    int nitems;
    void* fields;
    double* staging;
    double* diag_partial;
    double* diag_out;
    int64_t step;
    bool ready;
    tlb_launch launch;  // width, height = stream groups, chunk = rows per work item, variant
    // Stream groups: the domains are split over `groups` sets of nearly equal work, each stepped by
    // its own chain of launches on its own stream, forked from and joined back into `stream` by
    // events, so that one group's launch fills the compute units another's leaves idle while it
    // drains.  One group runs on `stream` itself.  The group streams are created together, the
    // first time more than one group is asked for, so that the runtime spreads them over distinct
    // hardware queues (streams that share a queue run one after the other).
    int groups;
    int grid[kMaxGroups];
    hipStream_t group_stream[kMaxGroups];
    hipEvent_t fork, join[kMaxGroups];
    int graph_steps;
    hipGraphExec_t graph_exec[kMaxGroups];
    hipGraph_t graph[kMaxGroups];
    std::vector<int64_t> wet_outside;  // [dom][wall]: wetting values with |4 h_m / (alpha kappa_m)| > 1
    bool wet_warned;
};

static thread_local int g_batch_last_hip = 0;

#define BHIP(...)                                                 \
    do {                                                          \
        hipError_t e_ = (__VA_ARGS__);                            \
        if (e_ != hipSuccess) {                                   \
            g_batch_last_hip = (int)e_;                           \
            return e_ == hipErrorOutOfMemory ? TLB_ENOMEM : TLB_EHIP; \
        }                                                         \
    } while (0)

template <typename T>
static Phys<T> phys_of(const tlb_params& p)
{
    Phys<T> P;
    const double a2 = p.alpha * p.alpha;
    for (int m = 0; m < 3; ++m) {
        P.kappa[m] = T(p.kappa[m]);
        P.a2kappa[m] = T(a2 * p.kappa[m]);
    }
    P.omega[0] = T(1.0 / p.tau_f);
    P.omega[1] = T(1.0 / p.tau_g);
    P.omega[2] = T(1.0 / p.tau_k);
    P.gphi3 = T(3.0 * p.gamma_phi);
    P.gpsi3 = T(3.0 * p.gamma_psi);
    P.adv = p.no_advection ? T(0) : T(1);
    P.mrt_sg = P.mrt_dv = P.mrt_db = T(0);
    return P;
}

static AuxGeom dom_geom(const tlb_batch* b, int d)
{
    AuxGeom g;
    g.lattice = 0;
    g.nx = b->p[d].nx;
    g.ny = b->p[d].ny;
    g.nz = 1;
    g.walls = b->p[d].walls_y;
    g.N = (int64_t)g.nx * g.ny;
    return g;
}

static void drop_graph(tlb_batch* b)
{
    for (int L = 0; L < kMaxGroups; ++L) {
        if (b->graph_exec[L]) (void)hipGraphExecDestroy(b->graph_exec[L]);
        if (b->graph[L]) (void)hipGraphDestroy(b->graph[L]);
        b->graph_exec[L] = nullptr;
        b->graph[L] = nullptr;
    }
}

// Waits for the work of every group's stream (the groups are joined into `stream` only at the end of
// tlb_batch_step, so a failed step can leave them running).
static hipError_t sync_groups(tlb_batch* b)
{
    hipError_t e = hipStreamSynchronize(b->stream);
    for (int L = 0; L < kMaxGroups; ++L)
        if (b->group_stream[L]) {
            const hipError_t f = hipStreamSynchronize(b->group_stream[L]);
            if (e == hipSuccess) e = f;
        }
    return e;
}

// Work items and queues for the current launch shape: domains go to the
// least-loaded stream group in decreasing size, then, within a group, to its
// least-loaded queue in decreasing size; within a queue, larger domains come
// first and the strips of one chunk are adjacent.  The flat items in the last
// quarter of a queue's work are halved, so that the workgroups run out of
// work at nearly the same time.
template <typename T>
static tlb_status build_items(tlb_batch* b)
{
    const int W = b->launch.width, rows = b->launch.chunk;
    std::vector<int> order(b->ndom);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        return (int64_t)b->p[a].nx * b->p[a].ny > (int64_t)b->p[c].nx * b->p[c].ny;
    });
    const int S = b->groups;
    std::vector<int> group_of(b->ndom);
    {
        std::vector<int64_t> gload(S, 0);
        for (int d : order) {
            const int L = (int)(std::min_element(gload.begin(), gload.end()) - gload.begin());
            group_of[d] = L;
            gload[L] += (int64_t)(b->p[d].nx + 2) * b->p[d].ny;
        }
    }
    auto flat_item = [](int d, int seg0, int cnt, bool down) {
        return make_int2(d, (int)((uint32_t)seg0 | (uint32_t)cnt << 16 | (down ? 0x80000000u : 0u)));
    };
    std::vector<DomDesc<T>> dd(b->ndom);
    std::vector<int2> items;
    std::vector<int> qs((size_t)kMaxGroups * (kQueues + 1), 0);
    std::vector<int> group_items(kMaxGroups, 0);
    for (int L = 0; L < S; ++L) {
        std::vector<std::vector<int2>> q(kQueues);
        std::vector<std::vector<int64_t>> qcost(kQueues);  // lane-rows of each item
        std::vector<int64_t> load(kQueues, 0);
        for (int d : order) {
            if (group_of[d] != L) continue;
            const tlb_params& p = b->p[d];
            DomDesc<T>& D = dd[d];
            D.off = b->off[d];
            D.wet_off = b->wet_off[d];
            D.nx = p.nx;
            D.ny = p.ny;
            D.walls = p.walls_y;
            D.P = phys_of<acc_t<T>>(p);
            const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            if (b->launch.variant == 2 && p.nx + 3 <= W) {
                // flat sweep: items of `rows` segments of W positions of the padded rows
                const int64_t nseg = ((int64_t)(p.nx + 2) * p.ny + W - 1) / W;
                D.flat = 1;
                D.chunk = (int)std::min<int64_t>(std::min(rows, 0x7fff), nseg);
                D.ntx = 1;
                D.nchunks = (int)((nseg + D.chunk - 1) / D.chunk);
                load[k] += nseg * W;
                for (int c = 0; c < D.nchunks; ++c) {
                    const int s0 = c * D.chunk, cnt = (int)std::min<int64_t>(D.chunk, nseg - s0);
                    q[k].push_back(flat_item(d, s0, cnt, c & 1));
                    qcost[k].push_back((int64_t)cnt * W);
                }
                continue;
            } else {
                D.flat = 0;
                D.chunk = std::min(rows, p.ny);
                D.ntx = (p.nx + W - 1) / W;
                D.nchunks = (p.ny + D.chunk - 1) / D.chunk;
                load[k] += (int64_t)D.ntx * W * p.ny;
            }
            for (int c = 0; c < D.nchunks; ++c)
                for (int s = 0; s < D.ntx; ++s) {
                    q[k].push_back(make_int2(d, (s << 16) | c));
                    qcost[k].push_back((int64_t)W * std::min(D.chunk, p.ny - c * D.chunk));
                }
        }
        for (int k = 0; k < kQueues; ++k) {
            int64_t total = 0, cum = 0;
            for (int64_t c : qcost[k]) total += c;
            std::vector<int2> split;
            for (size_t i = 0; i < q[k].size(); ++i) {
                const int2 it = q[k][i];
                const int cnt = (it.y >> 16) & 0x7fff;
                if (dd[it.x].flat && cnt >= 2 && 4 * cum >= 3 * total) {
                    const int s0 = it.y & 0xffff, h = cnt / 2;
                    const bool down = it.y < 0;
                    split.push_back(flat_item(it.x, s0, h, down));
                    split.push_back(flat_item(it.x, s0 + h, cnt - h, !down));
                } else {
                    split.push_back(it);
                }
                cum += qcost[k][i];
            }
            q[k].swap(split);
        }
        const int first = (int)items.size();
        for (int k = 0; k < kQueues; ++k) {
            qs[(size_t)L * (kQueues + 1) + k] = (int)items.size();
            items.insert(items.end(), q[k].begin(), q[k].end());
        }
        qs[(size_t)L * (kQueues + 1) + kQueues] = (int)items.size();
        group_items[L] = (int)items.size() - first;
    }
    if (b->items) BHIP(hipFree(b->items));
    b->items = nullptr;
    BHIP(hipMalloc((void**)&b->items, sizeof(int2) * items.size()));
    BHIP(hipMemcpyAsync(b->items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice, b->stream));
    BHIP(hipMemcpyAsync(b->qstart, qs.data(), sizeof(int) * qs.size(), hipMemcpyHostToDevice, b->stream));
    BHIP(hipMemcpyAsync(b->doms, dd.data(), sizeof(DomDesc<T>) * dd.size(), hipMemcpyHostToDevice, b->stream));
    BHIP(hipMemsetAsync(b->counters, 0, sizeof(int) * 2 * kQueues * kMaxGroups, b->stream));
    BHIP(hipStreamSynchronize(b->stream));
    b->nitems = (int)items.size();
    int dev = 0, ncu = 0, per_cu = 0;
    BHIP(hipGetDevice(&dev));
    BHIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    BHIP(occupancy_batch2d<T>(W, b->launch.variant, &per_cu));
    if (per_cu < 1) per_cu = 1;
    for (int L = 0; L < kMaxGroups; ++L) b->grid[L] = std::min(ncu * per_cu, group_items[L]);
    if (S > 1 && !b->group_stream[0]) {
        hipStream_t gs[kMaxGroups] = {};
        hipError_t e = hipSuccess;
        for (int L = 0; L < kMaxGroups && e == hipSuccess; ++L) e = hipStreamCreateWithFlags(&gs[L], hipStreamNonBlocking);
        if (e != hipSuccess) {  // all four or none
            for (hipStream_t x : gs)
                if (x) (void)hipStreamDestroy(x);
            BHIP(e);
        }
        for (int L = 0; L < kMaxGroups; ++L) b->group_stream[L] = gs[L];
    }
    drop_graph(b);
    return TLB_OK;
}

static tlb_status rebuild(tlb_batch* b)
{
    return b->prec == TLB_F32 ? build_items<float>(b) : build_items<double>(b);
}

extern "C" tlb_status tlb_batch_create(const tlb_params* per_dom, int32_t ndom, void* stream, tlb_batch** out)
{
    if (!per_dom || !out || ndom < 1) return TLB_EINVAL;
    *out = nullptr;
    const int prec = per_dom[0].prec;
    for (int d = 0; d < ndom; ++d) {
        const tlb_params& p = per_dom[d];
        if (p.lattice != TLB_D2Q9 || p.prec != prec || p.nz != 1) return TLB_EINVAL;
        if (p.nx < 3 || p.ny < 3 || p.nx > 65535 || p.ny > 65535 || (p.walls_y != 0 && p.walls_y != 1)) return TLB_EINVAL;
        for (int m = 0; m < 3; ++m)
            if (!(p.kappa[m] > 0.0) || !isfinite(p.kappa[m])) return TLB_EINVAL;
        if (!(p.alpha > 0.0) || !isfinite(p.alpha)) return TLB_EINVAL;
        if (!(p.tau_f > 0.5 && p.tau_g > 0.5 && p.tau_k > 0.5)) return TLB_EINVAL;
        if (!isfinite(p.tau_f) || !isfinite(p.tau_g) || !isfinite(p.tau_k)) return TLB_EINVAL;
        if (!isfinite(p.gamma_phi) || !isfinite(p.gamma_psi)) return TLB_EINVAL;
        if (p.no_advection != 0 && p.no_advection != 1) return TLB_EINVAL;
        if (p.collision != TLB_BGK) return TLB_EINVAL;  // the batched step collides with BGK
        if (p.ncomp != 0 && p.ncomp != 3) return TLB_EINVAL;  // and holds three components
        if (prec != TLB_F32 && prec != TLB_F64) return TLB_EINVAL;
        const int64_t bytes = (int64_t)27 * p.nx * p.ny * (prec == TLB_F32 ? 4 : 8);
        if (bytes > (int64_t)0xFFFFFF00) return TLB_EINVAL;
    }
    tlb_batch* b = new (std::nothrow) tlb_batch();
    if (!b) return TLB_ENOMEM;
    b->ndom = ndom;
    b->prec = prec;
    b->esize = prec == TLB_F32 ? 4 : 8;
    b->p.assign(per_dom, per_dom + ndom);
    b->off.resize(ndom);
    b->wet_off.resize(ndom);
    b->wet_outside.assign(2 * (size_t)ndom, 0);
    b->wet_warned = false;
    b->state_elems = b->wet_elems = b->total_nodes = b->max_nodes = 0;
    for (int d = 0; d < ndom; ++d) {
        const int64_t N = (int64_t)per_dom[d].nx * per_dom[d].ny;
        b->off[d] = b->state_elems;
        b->state_elems += ((27 * N + 63) / 64) * 64;  // 512-byte aligned domain blocks (FP64)
        b->wet_off[d] = per_dom[d].walls_y ? b->wet_elems : -1;
        if (per_dom[d].walls_y) b->wet_elems += 6 * (int64_t)per_dom[d].nx;
        b->total_nodes += N;
        b->max_nodes = std::max(b->max_nodes, N);
    }
    b->launch.width = 64;
    b->launch.height = 1;
    b->launch.chunk = 16;
    b->launch.variant = prec == TLB_F32 ? 1 : 0;
    b->groups = 1;
    hipError_t e = hipSuccess;
    if (stream) {
        b->stream = (hipStream_t)stream;
    } else {
        e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        b->own_stream = true;
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int L = 0; L < kMaxGroups && e == hipSuccess; ++L) e = hipEventCreateWithFlags(&b->join[L], hipEventDisableTiming);
    const size_t dsz = prec == TLB_F32 ? sizeof(DomDesc<float>) : sizeof(DomDesc<double>);
    if (e == hipSuccess) e = hipMalloc(&b->state[0], b->state_elems * b->esize);
    if (e == hipSuccess) e = hipMalloc(&b->state[1], b->state_elems * b->esize);
    if (e == hipSuccess) e = hipMalloc(&b->wet, std::max<int64_t>(b->wet_elems, 1) * b->esize);
    if (e == hipSuccess) e = hipMemsetAsync(b->wet, 0, std::max<int64_t>(b->wet_elems, 1) * b->esize, b->stream);
    if (e == hipSuccess) e = hipMalloc(&b->doms, dsz * ndom);
    if (e == hipSuccess) e = hipMalloc((void**)&b->qstart, sizeof(int) * kMaxGroups * (kQueues + 1));
    if (e == hipSuccess) e = hipMalloc((void**)&b->counters, sizeof(int) * kMaxGroups * 2 * kQueues);
    if (e == hipSuccess) e = hipMalloc((void**)&b->diag_partial, sizeof(double) * kDiagBlocks * kDiagSlots);
    if (e == hipSuccess) e = hipMalloc((void**)&b->diag_out, sizeof(double) * kDiagSlots);
    if (e != hipSuccess) {
        g_batch_last_hip = (int)e;
        tlb_batch_destroy(b);
        return e == hipErrorOutOfMemory ? TLB_ENOMEM : TLB_EHIP;
    }
    tlb_status st = rebuild(b);
    if (st) {
        tlb_batch_destroy(b);
        return st;
    }
    *out = b;
    return TLB_OK;
}

extern "C" tlb_status tlb_batch_destroy(tlb_batch* b)
{
    if (!b) return TLB_EINVAL;
    (void)sync_groups(b);
    drop_graph(b);
    for (void* ptr : {b->state[0], b->state[1], b->wet, b->doms, (void*)b->items, (void*)b->qstart, (void*)b->counters,
                      b->fields, (void*)b->staging, (void*)b->diag_partial, (void*)b->diag_out})
        if (ptr) (void)hipFree(ptr);
    for (int L = 0; L < kMaxGroups; ++L) {
        if (b->group_stream[L]) (void)hipStreamDestroy(b->group_stream[L]);
        if (b->join[L]) (void)hipEventDestroy(b->join[L]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return TLB_OK;
}

extern "C" int32_t tlb_batch_size(const tlb_batch* b) { return b ? b->ndom : 0; }
extern "C" int64_t tlb_batch_nodes(const tlb_batch* b) { return b ? b->total_nodes : 0; }
extern "C" void* tlb_batch_get_stream(const tlb_batch* b) { return b ? (void*)b->stream : nullptr; }

extern "C" tlb_status tlb_batch_synchronize(tlb_batch* b)
{
    if (!b) return TLB_EINVAL;
    BHIP(hipStreamSynchronize(b->stream));
    return TLB_OK;
}

static tlb_status staging(tlb_batch* b)
{
    if (b->staging) return TLB_OK;
    BHIP(hipMalloc((void**)&b->staging, sizeof(double) * 27 * b->max_nodes));
    return TLB_OK;
}

extern "C" tlb_status tlb_batch_set_wetting(tlb_batch* b, int32_t dom, int wall, const double* h)
{
    if (!b || !h || dom < 0 || dom >= b->ndom || (wall != 0 && wall != 1) || !b->p[dom].walls_y) return TLB_EINVAL;
    const tlb_params& p = b->p[dom];
    for (int j = 0; j < 3 * p.nx; ++j)
        if (!isfinite(h[j])) return TLB_EINVAL;
    // values outside the closed-form range of the wall free energy (Sec. II.B) are applied as
    // given; they are counted and reported once per batch on stderr
    int64_t outside = 0;
    for (int m = 0; m < 3; ++m)
        for (int j = 0; j < p.nx; ++j) outside += fabs(h[m * p.nx + j]) > 0.25 * p.alpha * p.kappa[m];
    b->wet_outside[2 * (size_t)dom + wall] = outside;
    if (outside > 0 && !b->wet_warned) {
        b->wet_warned = true;
        fprintf(stderr,
                "libtlb: warning: domain %d, wall %d: %lld wetting parameters have |4 h_m / (alpha kappa_m)| > 1, "
                "outside the range of the closed-form wall concentrations and contact angles (Sec. II.B); the "
                "boundary condition is still applied as given (further domains are not reported; see "
                "tlb_batch_wetting_outside_range)\n",
                dom, wall, (long long)outside);
    }
    tlb_status st = staging(b);
    if (st) return st;
    BHIP(hipMemcpyAsync(b->staging, h, sizeof(double) * 3 * p.nx, hipMemcpyHostToDevice, b->stream));
    const double a2 = p.alpha * p.alpha;
    const int64_t o = b->wet_off[dom] + (int64_t)wall * 3 * p.nx;
    const WetScale inv = {{1.0 / (a2 * p.kappa[0]), 1.0 / (a2 * p.kappa[1]), 1.0 / (a2 * p.kappa[2])}};
    if (b->prec == TLB_F32)
        BHIP(launch_wet<float, double>(p.nx, 3, b->staging, inv, (float*)b->wet + o, b->stream));
    else
        BHIP(launch_wet<double, double>(p.nx, 3, b->staging, inv, (double*)b->wet + o, b->stream));
    BHIP(hipStreamSynchronize(b->stream));
    return TLB_OK;
}

extern "C" tlb_status tlb_batch_wetting_outside_range(const tlb_batch* b, int32_t dom, int64_t* count)
{
    if (!b || !count || dom < -1 || dom >= b->ndom) return TLB_EINVAL;
    int64_t c = 0;
    for (int d = (dom < 0 ? 0 : dom); d < (dom < 0 ? b->ndom : dom + 1); ++d)
        c += b->wet_outside[2 * (size_t)d] + b->wet_outside[2 * (size_t)d + 1];
    *count = c;
    return TLB_OK;
}

extern "C" tlb_status tlb_batch_init_equilibrium(tlb_batch* b, int32_t dom, const double* C, const double* u)
{
    if (!b || !C || dom < 0 || dom >= b->ndom) return TLB_EINVAL;
    const AuxGeom g = dom_geom(b, dom);
    tlb_status st = staging(b);
    if (st) return st;
    BHIP(hipMemcpyAsync(b->staging, C, sizeof(double) * 3 * g.N, hipMemcpyHostToDevice, b->stream));
    const double* ud = nullptr;
    if (u) {
        BHIP(hipMemcpyAsync(b->staging + 3 * g.N, u, sizeof(double) * 2 * g.N, hipMemcpyHostToDevice, b->stream));
        ud = b->staging + 3 * g.N;
    }
    if (b->prec == TLB_F32)
        BHIP(launch_init<float, double>(g, phys_of<acc_t<float>>(b->p[dom]), b->staging, ud,
                                        b->wet_off[dom] >= 0 ? (const float*)b->wet + b->wet_off[dom] : nullptr,
                                        (float*)b->state[b->cur] + b->off[dom], b->stream));
    else
        BHIP(launch_init<double, double>(g, phys_of<acc_t<double>>(b->p[dom]), b->staging, ud,
                                         b->wet_off[dom] >= 0 ? (const double*)b->wet + b->wet_off[dom] : nullptr,
                                         (double*)b->state[b->cur] + b->off[dom], b->stream));
    BHIP(hipStreamSynchronize(b->stream));
    b->ready = true;
    b->step = 0;
    return TLB_OK;
}

// The stream group L runs on: `stream` itself when there is one group.
static hipStream_t gstream(const tlb_batch* b, int L) { return b->groups > 1 ? b->group_stream[L] : b->stream; }

// One step of stream group L from buffer `cur` on the group's stream.
template <typename T>
static tlb_status batch_launch_one(tlb_batch* b, int L, int cur)
{
    BatchArgs<T> a;
    a.src = (const T*)b->state[cur];
    a.dst = (T*)b->state[cur ^ 1];
    a.wet = (const T*)b->wet;
    a.doms = (const DomDesc<T>*)b->doms;
    a.items = b->items;
    a.qstart = b->qstart + L * (kQueues + 1);
    a.counters = b->counters + L * 2 * kQueues;
    a.parity = cur;
    BHIP(launch_batch2d<T>(a, b->launch.width, b->launch.variant, b->grid[L], gstream(b, L)));
    return TLB_OK;
}

static tlb_status launch_one(tlb_batch* b, int L, int cur)
{
    return b->prec == TLB_F32 ? batch_launch_one<float>(b, L, cur) : batch_launch_one<double>(b, L, cur);
}

// The groups' streams wait for the work queued on `stream` so far.
static tlb_status fork_groups(tlb_batch* b)
{
    if (b->groups < 2) return TLB_OK;
    BHIP(hipEventRecord(b->fork, b->stream));
    for (int L = 0; L < b->groups; ++L) BHIP(hipStreamWaitEvent(b->group_stream[L], b->fork, 0));
    return TLB_OK;
}

// Work queued on `stream` from now on waits for the groups' streams.
static tlb_status join_groups(tlb_batch* b)
{
    if (b->groups < 2) return TLB_OK;
    for (int L = 0; L < b->groups; ++L) {
        BHIP(hipEventRecord(b->join[L], b->group_stream[L]));
        BHIP(hipStreamWaitEvent(b->stream, b->join[L], 0));
    }
    return TLB_OK;
}

// n steps of every group, step by step across the groups so that all streams are fed.
static tlb_status launch_steps(tlb_batch* b, int64_t n)
{
    for (int64_t t = 0; t < n; ++t) {
        for (int L = 0; L < b->groups; ++L) {
            tlb_status st = launch_one(b, L, b->cur);
            if (st) return st;
        }
        b->cur ^= 1;
    }
    return TLB_OK;
}

static tlb_status batch_direct(tlb_batch* b, int64_t n)
{
    tlb_status st = fork_groups(b);
    if (!st) st = launch_steps(b, n);
    if (!st) st = join_groups(b);
    return st;
}

extern "C" tlb_status tlb_batch_step(tlb_batch* b, int64_t nsteps)
{
    if (!b || nsteps < 0) return TLB_EINVAL;
    if (!b->ready) return TLB_ESTATE;
    int64_t left = nsteps;
    tlb_status st = fork_groups(b);
    if (st) return st;
    if (b->graph_steps > 0 && left >= b->graph_steps) {
        if (b->cur != 0) {  // the captured chains start from buffer 0
            st = launch_steps(b, 1);
            if (st) return st;
            --left;
        }
        // one captured chain per group, on the group's stream
        for (int L = 0; L < b->groups; ++L) {
            if (b->graph_exec[L]) continue;
            hipStream_t s = gstream(b, L);
            BHIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            for (int t = 0; t < b->graph_steps && !st; ++t) st = launch_one(b, L, t & 1);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(s, &g);
            if (st) return st;
            BHIP(e);
            b->graph[L] = g;
            BHIP(hipGraphInstantiate(&b->graph_exec[L], g, nullptr, nullptr, 0));
        }
        while (left >= b->graph_steps) {
            for (int L = 0; L < b->groups; ++L) BHIP(hipGraphLaunch(b->graph_exec[L], gstream(b, L)));
            left -= b->graph_steps;
        }
    }
    st = launch_steps(b, left);
    if (!st) st = join_groups(b);
    if (st) return st;
    b->step += nsteps;
    return TLB_OK;
}

extern "C" tlb_status tlb_batch_set_graph(tlb_batch* b, int32_t steps_per_graph)
{
    if (!b || steps_per_graph < 0 || (steps_per_graph & 1)) return TLB_EINVAL;
    BHIP(sync_groups(b));
    drop_graph(b);
    b->graph_steps = steps_per_graph;
    return TLB_OK;
}

extern "C" tlb_status tlb_batch_set_launch(tlb_batch* b, const tlb_launch* l)
{
    if (!b || !l) return TLB_EINVAL;
    if ((l->width != 64 && l->width != 128 && l->width != 256) || l->chunk < 1 || l->chunk > 65535 ||
        l->variant < 0 || l->variant > 2 || l->height < 0 || l->height > kMaxGroups)
        return TLB_EINVAL;
    BHIP(sync_groups(b));
    const tlb_launch old = b->launch;
    const int old_groups = b->groups;
    b->launch = *l;
    b->groups = std::max(1, std::min(l->height, b->ndom));
    b->launch.height = b->groups;
    const tlb_status st = rebuild(b);
    if (st) {  // keep the batch steppable in its previous shape
        b->launch = old;
        b->groups = old_groups;
        (void)rebuild(b);
    }
    return st;
}

extern "C" tlb_status tlb_batch_get_launch(const tlb_batch* b, tlb_launch* out)
{
    if (!b || !out) return TLB_EINVAL;
    *out = b->launch;
    return TLB_OK;
}

extern "C" tlb_status tlb_batch_get_field(tlb_batch* b, int32_t dom, int which, double* out)
{
    if (!b || !out || dom < 0 || dom >= b->ndom || which < 0 || which >= TLB_NFIELDS) return TLB_EINVAL;
    if (!b->ready) return TLB_ESTATE;
    const AuxGeom g = dom_geom(b, dom);
    tlb_status st = staging(b);
    if (st) return st;
    if (!b->fields) BHIP(hipMalloc(&b->fields, (size_t)TLB_NFIELDS * b->max_nodes * b->esize));
    if (b->prec == TLB_F32) {
        const float* wet = b->wet_off[dom] >= 0 ? (const float*)b->wet + b->wet_off[dom] : nullptr;
        BHIP(launch_fields<float>(g, phys_of<acc_t<float>>(b->p[dom]), (const float*)b->state[b->cur] + b->off[dom], wet,
                                  (float*)b->fields, b->stream));
        BHIP(launch_export_field<float, double>(g, (const float*)b->fields, which, b->staging, b->stream));
    } else {
        const double* wet = b->wet_off[dom] >= 0 ? (const double*)b->wet + b->wet_off[dom] : nullptr;
        BHIP(launch_fields<double>(g, phys_of<acc_t<double>>(b->p[dom]), (const double*)b->state[b->cur] + b->off[dom], wet,
                                   (double*)b->fields, b->stream));
        BHIP(launch_export_field<double, double>(g, (const double*)b->fields, which, b->staging, b->stream));
    }
    BHIP(hipMemcpyAsync(out, b->staging, sizeof(double) * g.N, hipMemcpyDeviceToHost, b->stream));
    BHIP(hipStreamSynchronize(b->stream));
    return TLB_OK;
}

extern "C" tlb_status tlb_batch_get_populations(tlb_batch* b, int32_t dom, int species, double* out)
{
    if (!b || !out || dom < 0 || dom >= b->ndom || species < 0 || species > 2) return TLB_EINVAL;
    if (!b->ready) return TLB_ESTATE;
    const AuxGeom g = dom_geom(b, dom);
    tlb_status st = staging(b);
    if (st) return st;
    if (b->prec == TLB_F32)
        BHIP(launch_get_pops<float, double>(g, (const float*)b->state[b->cur] + b->off[dom], species, b->staging,
                                            b->stream));
    else
        BHIP(launch_get_pops<double, double>(g, (const double*)b->state[b->cur] + b->off[dom], species, b->staging,
                                             b->stream));
    BHIP(hipMemcpyAsync(out, b->staging, sizeof(double) * 9 * g.N, hipMemcpyDeviceToHost, b->stream));
    BHIP(hipStreamSynchronize(b->stream));
    return TLB_OK;
}

extern "C" tlb_status tlb_batch_diagnostics(tlb_batch* b, int32_t dom, tlb_diag* out)
{
    if (!b || !out || dom < 0 || dom >= b->ndom) return TLB_EINVAL;
    if (!b->ready) return TLB_ESTATE;
    const AuxGeom g = dom_geom(b, dom);
    if (b->prec == TLB_F32)
        BHIP(launch_diag<float>(g, (const float*)b->state[b->cur] + b->off[dom], b->diag_partial, kDiagBlocks,
                                b->diag_out, b->stream));
    else
        BHIP(launch_diag<double>(g, (const double*)b->state[b->cur] + b->off[dom], b->diag_partial, kDiagBlocks,
                                 b->diag_out, b->stream));
    double h[kDiagSlots];
    BHIP(hipMemcpyAsync(h, b->diag_out, sizeof(h), hipMemcpyDeviceToHost, b->stream));
    BHIP(hipStreamSynchronize(b->stream));
    for (int m = 0; m < 3; ++m) {
        out->mass[m] = h[m];
        out->momentum[m] = h[3 + m];
        out->interface[m] = h[8 + m];
    }
    out->max_speed = h[6];
    out->nonfinite = (int64_t)h[7];
    out->step = b->step;
    return out->nonfinite ? TLB_ENAN : TLB_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: times every launch shape for a few steps from the current state
// (restored afterwards) and keeps the fastest.  With the environment variable
// TLB_TUNE_CACHE naming a file, results are looked up there first and new
// ones appended, keyed by the batch's shape signature.
// ---------------------------------------------------------------------------
static std::string batch_signature(const tlb_batch* b)
{
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the domain sizes and walls
    for (const tlb_params& p : b->p) {
        const uint64_t v[3] = {(uint64_t)p.nx, (uint64_t)p.ny, (uint64_t)p.walls_y};
        for (uint64_t x : v)
            for (int k = 0; k < 8; ++k) {
                h ^= (x >> (8 * k)) & 0xff;
                h *= 1099511628211ull;
            }
    }
    char buf[128];
    snprintf(buf, sizeof(buf), "batch-d2q9-%s-%d-%llx", b->prec == TLB_F32 ? "f32" : "f64", b->ndom,
             (unsigned long long)h);
    return buf;
}

// Cache lines: key width chunk variant groups (lines with fewer fields are skipped).
static bool cache_lookup(const char* path, const std::string& key, tlb_launch* l)
{
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[256], k[128];
    int w, c, v, g;
    bool found = false;
    while (fgets(line, sizeof(line), f))
        if (sscanf(line, "%127s %d %d %d %d", k, &w, &c, &v, &g) == 5 && key == k) {
            l->width = w;
            l->height = g;
            l->chunk = c;
            l->variant = v;
            found = true;
        }
    fclose(f);
    return found;
}

extern "C" tlb_status tlb_batch_autotune(tlb_batch* b, int32_t trial_steps, tlb_launch* chosen)
{
    if (!b || trial_steps < 1) return TLB_EINVAL;
    if (!b->ready) return TLB_ESTATE;
    const char* cache = getenv("TLB_TUNE_CACHE");
    const std::string key = batch_signature(b);
    tlb_launch best;
    if (cache && cache_lookup(cache, key, &best)) {
        tlb_status st = tlb_batch_set_launch(b, &best);
        if (st) return st;
        if (chosen) *chosen = best;
        return TLB_OK;
    }
    BHIP(hipStreamSynchronize(b->stream));
    const size_t bytes = (size_t)b->state_elems * b->esize;
    void* save = nullptr;
    BHIP(hipMalloc(&save, bytes));
    const int cur0 = b->cur;
    const int gsave = b->graph_steps;
    b->graph_steps = 0;
    hipEvent_t e0, e1;
    BHIP(hipEventCreate(&e0));
    BHIP(hipEventCreate(&e1));
    BHIP(hipMemcpyAsync(save, b->state[cur0], bytes, hipMemcpyDeviceToDevice, b->stream));
    float best_ms = 1e30f;
    best = b->launch;
    const int widths[3] = {64, 128, 256};
    const int chunks[4] = {8, 16, 32, 64};
    tlb_status st = TLB_OK;
    float margin = 1.0f;  // a later shape replaces the best one if its time is below margin * best
    auto trial = [&](const tlb_launch& l, int steps) {
        st = tlb_batch_set_launch(b, &l);
        // warm-up as long as the trial: a group's first launches on a new stream are slower
        if (!st) st = batch_direct(b, steps);
        if (st) return;
        (void)hipEventRecord(e0, b->stream);
        st = batch_direct(b, steps);
        (void)hipEventRecord(e1, b->stream);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (!st && ms < margin * best_ms) {
            best_ms = ms;
            best = l;
        }
    };
    // every shape in one stream group; then the fastest of them again in 1..4 groups and with items of
    // one, two and four times its rows (with several groups the drain of one launch is covered by the
    // others, so longer items, with fewer halo rows, can pay), with four times the steps (these
    // differ by a few percent)
    for (int wi = 0; wi < 3 && !st; ++wi)
        for (int ci = 0; ci < 4 && !st; ++ci)
            for (int v = 0; v < 3 && !st; ++v) trial(tlb_launch{widths[wi], 1, chunks[ci], v}, trial_steps);
    const tlb_launch one = best;
    best_ms = 1e30f;
    margin = 0.995f;  // fewer groups and shorter items first; a later one must be faster by more than 0.5%
    for (int g = 1; g <= std::min(kMaxGroups, b->ndom) && !st; ++g)
        for (int f = 1; f <= 4 && !st; f *= 2)
            if ((int64_t)one.chunk * f <= 65535) trial(tlb_launch{one.width, g, one.chunk * f, one.variant}, 4 * trial_steps);
    (void)hipMemcpyAsync(b->state[cur0], save, bytes, hipMemcpyDeviceToDevice, b->stream);
    (void)hipStreamSynchronize(b->stream);
    (void)hipFree(save);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->cur = cur0;
    b->graph_steps = gsave;
    if (st) return st;
    st = tlb_batch_set_launch(b, &best);
    if (st) return st;
    if (cache) {
        FILE* f = fopen(cache, "a");
        if (f) {
            fprintf(f, "%s %d %d %d %d\n", key.c_str(), best.width, best.chunk, best.variant, best.height);
            fclose(f);
        }
    }
    if (chosen) *chosen = best;
    return TLB_OK;
}
