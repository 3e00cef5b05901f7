// The fused time-step kernel and its launchers, instantiated once per store
// format (step_f64.hip, step_f32.hip, step_f16.hip, step_bf16.hip).
//
// Method: Han, Ooka & Kikumoto, "A wall function approach in lattice
// Boltzmann method" (arXiv 2009.04352).  One kernel launch per time step
// does, for every cell: streaming (Eq. 1) with wall reflections (bounce-back,
// Eq. 3 in 3-D form; mirror reflection, Eq. 4 in 3-D form), the wall-function
// bounce correction at wall-adjacent cells (Eq. 13-17, Newton on Spalding's
// law in FP64), moments (Eq. 2), a Smagorinsky eddy viscosity from the local
// non-equilibrium stress (Sec. 3.1), BGK relaxation and the body force term
// F_a of Eq. 1.
//
// Streaming is the in-place "AA" pattern: a single population array; the
// odd kernel pulls from neighbours and pushes to neighbours, the even kernel
// reads and writes the cell's own slots.  Layouts between steps:
//   after an even number of steps ("P"): slot opp(a) of cell c holds the
//     post-collision f*_a(c);
//   after an odd number ("S"): slot a of cell c holds f_a(c) streamed in for
//     the next collision, wall-crossing links already reflected.
// Every odd-kernel work-item reads exactly the 19 slots it later writes, so
// the in-place update has no inter-thread hazards, walls included: a mirror
// read of slot opp(mirror a) at c - e_a^par is the slot the same cell writes
// its outgoing mirror(b) population to, b = opp(a).
#pragma once
#include <type_traits>

#include "lbm_device.h"

namespace lbmwf {

// Directions with a streamwise component: the only ones whose odd-step source
// and destination are shifted along x.  Each has an exchange slot in LDS.
constexpr int kNX = 10;
constexpr int xslot(int a)
{
    int j = 0;
    for (int b = 0; b < kQ; ++b)
        if (kEx[b] != 0) {
            if (b == a) return j;
            ++j;
        }
    return -1;
}

// The group [last element of nb, v0 .. v(V-2)] and [v1 .. v(V-1), first of nb].
template <typename S, int V>
__device__ __forceinline__ u32x2 join_left(u32x2 v, u32x2 nb)
{
    if constexpr (V == 1) return nb;
    else return Lane<S, V>::shift_in_left(v, Lane<S, V>::last(nb));
}
template <typename S, int V>
__device__ __forceinline__ u32x2 join_right(u32x2 v, u32x2 nb)
{
    if constexpr (V == 1) return nb;
    else return Lane<S, V>::shift_in_right(v, Lane<S, V>::first(nb));
}

// One element read straight from memory, placed as the last (first) element of a group.
template <typename S, int V>
__device__ __forceinline__ u32x2 halo_as_last(const typename S::T* p)
{
    using Ln = Lane<S, V>;
    if constexpr (V == 1) return Ln::template load<false>(p);
    else return Ln::as_last(Ln::load_elem(p));
}
template <typename S, int V>
__device__ __forceinline__ u32x2 halo_as_first(const typename S::T* p)
{
    using Ln = Lane<S, V>;
    if constexpr (V == 1) return Ln::template load<false>(p);
    else return Ln::as_first(Ln::load_elem(p));
}

// a3 for the V cells of a wall-row group: decode, the gathered wall-parallel
// velocity of each cell, the Newton solve for each friction velocity, and
// the half stresses hx = tau_x / 2, hz = tau_z / 2 that the bounce
// correction adds.  Wall rows are whole rows, so the branch that calls
// this is uniform over the wavefront.
template <typename S, int V>
__device__ __forceinline__ void wall_group(const u32x2 (&w)[kQ], const StepArgs& p, typename S::R (&hx)[V],
                                           typename S::R (&hz)[V], int& iters, bool& fail)
{
    using R = typename S::R;
    using Ln = Lane<S, V>;
    R rho[V], vx[V], vz[V];
    double U[V], ut[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
        R f[kQ];
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            f[a] = Ln::get(w[a], k);
        });
        U[k] = wall_velocity<R>(f, (R)p.fx, rho[k], vx[k], vz[k]);
    }
    // With 4 cells per thread: one solve per cell, in a loop kept rolled, so
    // that the solve's code appears once (unrolled over the 4 cells, or two
    // at a time, the odd step ran 2-5 % slower on MI355X).  With 1 or 2
    // cells the solves run side by side (rolled, the 2-cell kernels need
    // more registers).
    if constexpr (V < 4) {
        wall_utau_n<V>(U, p.y1, p.nu0, p.kappa, p.bconst, p.ekb, p.newton_tol, p.newton_maxit, ut, iters, fail);
    } else {
        iters = 0;
        fail = false;
#pragma unroll 1
        for (int k = 0; k < V; ++k) {
            double u1[1] = {U[0]}, t1[1];
#pragma unroll
            for (int j = 1; j < V; ++j)
                if (k == j) u1[0] = U[j];
            int it;
            bool fl;
            wall_utau_n<1>(u1, p.y1, p.nu0, p.kappa, p.bconst, p.ekb, p.newton_tol, p.newton_maxit, t1, it, fl);
            iters = max(iters, it);
            fail = fail || fl;
#pragma unroll
            for (int j = 0; j < V; ++j)
                if (k == j) ut[j] = t1[0];
        }
    }
#pragma unroll
    for (int k = 0; k < V; ++k) {
        const WallRecord rec = wall_record((double)rho[k], (double)vx[k], (double)vz[k], U[k], ut[k]);
        hx[k] = (R)(0.5 * rec.taux);
        hz[k] = (R)(0.5 * rec.tauz);
    }
}

// a3-a6 for the V cells of a group in place: decode, wall-function bounce
// (wall_wfb: the cells are wall-adjacent and the boundary is WFB), moments,
// Smagorinsky, BGK with the body force, encode.  Accumulates the sampled
// velocity sums, the largest Newton iteration count and the failure flags.
template <typename S, int V, bool MAYBE_WFB, bool STATS, bool MRT>
__device__ __forceinline__ void collide_group(u32x2 (&w)[kQ], const StepArgs& p, typename S::R cs2, bool wall_wfb,
                                              bool top, double (&sm)[7], int& iters, bool& bad, bool& newton_fail)
{
    using R = typename S::R;
    using Ln = Lane<S, V>;
    constexpr bool PAIRS = (sizeof(typename S::T) == 2) && (V >= 2);
    MrtRates<R> mr;
    if constexpr (MRT) {
#pragma unroll
        for (int i = 0; i < 5; ++i) mr.s[i] = (R)p.mrt_s[i];
    }
    // a3: wall-function bounce at wall-adjacent cells
    R whx[V], whz[V];
    if constexpr (MAYBE_WFB) {
        if (wall_wfb) {
            int it = 0;
            bool fail = false;
            wall_group<S, V>(w, p, whx, whz, it, fail);
            iters = max(iters, it);
            newton_fail = newton_fail || fail;
        }
    }
    auto cell = [&](int k, R (&f)[kQ]) {
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            f[a] = Ln::get(w[a], k);
        });
        if constexpr (MAYBE_WFB) {
            if (wall_wfb) wfb_apply<R>(f, top, whx[k], whz[k]);
        }
        // a4-a6: moments, Smagorinsky, BGK (or MRT) + body force
        const Moments<R> m = collide<R, MRT>(f, (R)p.tau0, cs2, (R)p.fx, &mr);
        bad = bad || !(m.rho > R(0)) || !(m.rho < R(INFINITY));
        if constexpr (STATS) {
            const double ux = (double)m.ux, uy = (double)m.uy, uz = (double)m.uz;
            sm[0] += ux; sm[1] += uy; sm[2] += uz;
            sm[3] += ux * ux; sm[4] += uy * uy; sm[5] += uz * uz; sm[6] += ux * uy;
        }
    };
    if constexpr (PAIRS) {
        // 2-byte stores: two cells are encoded by one packed conversion
#pragma unroll
        for (int k = 0; k < V; k += 2) {
            R f0[kQ], f1[kQ];
            cell(k, f0);
            cell(k + 1, f1);
            for_each_dir([&](auto A) {
                constexpr int a = decltype(A)::value;
                Ln::set_pair(w[a], k, f0[a], f1[a]);
            });
        }
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            R f[kQ];
            cell(k, f);
            for_each_dir([&](auto A) {
                constexpr int a = decltype(A)::value;
                Ln::set(w[a], k, f[a]);
            });
        }
    }
}

// Boundary of a launch: fixed at compile time for a single channel, read
// from the instance table for batched launches (instances differ).
constexpr int kBCRuntime = 3;

// ------------------------------------------------------------ wall nodes
//
// The wall grid of Sec. 2.1-2.2 taken literally: a lattice node one spacing
// outside each wall layer of fluid (y = -1 and y = ny), where the reflection
// happens (bounce-back, Eq. 3; mirror reflection, Eq. 4; WFB, Eq. 14).  A
// population the first layer sends towards the wall reaches the wall node
// of its column x + e_b one step later, is reflected there with the stress
// of Eq. 15-17 from the first layer's velocity of that (previous) step, and
// streams into the first layer at x + e_b + e_a one step after that: a lag of
// one step and twice the tangential shift of the halfway walls.  The kernel
// of the first-layer cell at column (x, z) also does the wall node's
// collision at (x, z); the rings that carry the populations in flight are
// described at wn_index.  (kBCNode: the reflection, StepArgs::bc, is read at
// run time.)
constexpr int kBCNode = 4;
// element k of a wall node holding direction A, which enters the fluid from wall `top`
template <int A>
__device__ __forceinline__ int node_k(bool top)
{
    return top ? in_index_b(mirror_y(A)) : in_index_b(A);
}

__device__ __forceinline__ int wrap_x(int x, int nx) { return x < 0 ? x + nx : (x >= nx ? x - nx : x); }

// The group of cells x0 .. x0 + V - 1 of a ring row, shifted by sh (the
// elements x0 + j + sh, x periodic).
template <typename S, int V>
__device__ __forceinline__ u32x2 ring_load(const typename S::T* row, int x0, int sh, int nx)
{
    using Ln = Lane<S, V>;
    if (sh == 0) return Ln::template load<false>(row + x0);
    if constexpr (V == 1) {
        return Ln::template load<false>(row + wrap_x(x0 + sh, nx));
    } else {
        unsigned int e[V];
#pragma unroll
        for (int j = 0; j < V; ++j) e[j] = Ln::load_elem(row + wrap_x(x0 + j + sh, nx));
        return Ln::from_elems(e);
    }
}

template <typename S, int V>
__device__ __forceinline__ void ring_store(typename S::T* row, int x0, int sh, int nx, u32x2 g)
{
    using Ln = Lane<S, V>;
    if (sh == 0) {
        Ln::template store<false>(row + x0, g);
        return;
    }
    if constexpr (V == 1) {
        Ln::template store<false>(row + wrap_x(x0 + sh, nx), g);
    } else {
#pragma unroll
        for (int j = 0; j < V; ++j) Ln::store_elem(row + wrap_x(x0 + j + sh, nx), Ln::elem(g, j));
    }
}

template <typename S>
__device__ __forceinline__ typename S::T* ring_row(const StepArgs& p, int ring, int wl, int k, int zz)
{
    return (typename S::T*)p.wn + wn_index(ring, wl, k, zz, 0, p.nx, p.nz);
}

// The wall-node collision of the V nodes below (above) this thread's cells:
// the arrivals of the previous step (ring `prev`) reflected by the boundary
// p.bc, with +-tau/2 on the four diagonals for WFB (Eq. 14a-b; tau from the
// first layer's record of the previous step, Eq. 15-17), into output ring
// 2 + cur.
template <typename S, int V>
__device__ __forceinline__ void node_collide(const StepArgs& p, bool top, int z, int x0, int prev, int cur)
{
    using R = typename S::R;
    using Ln = Lane<S, V>;
    const int wl = top ? 1 : 0;
    const bool wfb = (p.bc == kWFB), bb = (p.bc == kBB);
    R hx[V], hz[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
        hx[j] = R(0);
        hz[j] = R(0);
        if (wfb) {
            const double* r = p.wn_rec + (((long long)wl * p.nz + z) * p.nx + x0 + j) * 4;
            const double rho = r[0], ux = r[1], uz = r[2], ut = r[3];
            const double U = sqrt(ux * ux + uz * uz);
            const WallRecord rec = wall_record(rho, ux, uz, U, ut);
            hx[j] = (R)(0.5 * rec.taux);
            hz[j] = (R)(0.5 * rec.tauz);
        }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int ka = bb ? k : node_spec(k);
        u32x2 g = Ln::template load<false>(ring_row<S>(p, prev, wl, ka, z) + x0);
        if (wfb && k > 0) {
            // k = 1, 3: +-tau_x / 2 (directions 7, 14); k = 2, 4: +-tau_z / 2 (11, 17)
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const R d = (k == 1) ? hx[j] : (k == 3) ? -hx[j] : (k == 2) ? hz[j] : -hz[j];
                Ln::set(g, j, Ln::get(g, j) + d);
            }
        }
        Ln::template store<false>(ring_row<S>(p, 2 + cur, wl, k, z) + x0, g);
    }
}

// The record of the first-layer cells for the next wall-node collision:
// density, wall-parallel velocity and the friction velocity of Spalding's law
// (solved in FP64 as for the halfway walls), one solve per cell.
template <int V>
__device__ __forceinline__ void node_record(const StepArgs& p, bool top, int z, int x0, const double (&rho)[V],
                                            const double (&ux)[V], const double (&uz)[V], int& iters, bool& fail)
{
    double U[V], ut[V];
#pragma unroll
    for (int j = 0; j < V; ++j) U[j] = sqrt(ux[j] * ux[j] + uz[j] * uz[j]);
    iters = 0;
    fail = false;
#pragma unroll 1
    for (int j = 0; j < V; ++j) {
        double u1[1] = {U[0]}, t1[1];
#pragma unroll
        for (int i = 1; i < V; ++i)
            if (j == i) u1[0] = U[i];
        int it;
        bool fl;
        wall_utau_n<1>(u1, p.y1, p.nu0, p.kappa, p.bconst, p.ekb, p.newton_tol, p.newton_maxit, t1, it, fl);
        iters = max(iters, it);
        fail = fail || fl;
#pragma unroll
        for (int i = 0; i < V; ++i)
            if (j == i) ut[i] = t1[0];
    }
    const int wl = top ? 1 : 0;
#pragma unroll
    for (int j = 0; j < V; ++j) {
        double* r = p.wn_rec + (((long long)wl * p.nz + z) * p.nx + x0 + j) * 4;
        r[0] = rho[j];
        r[1] = ux[j];
        r[2] = uz[j];
        r[3] = ut[j];
    }
}

// One time step for V consecutive cells per thread.  A block holds one tile
// of an instance: either `rpb` whole x-rows of one z-plane (nx / V threads
// per row) or one segment of a single x-row (tile_x threads).  Every global
// access is an aligned V-element group.  In the odd step the x-shifted
// directions exchange neighbouring elements through LDS: a thread takes the
// element it lacks from its neighbour in the row segment; a whole row wraps
// around inside the block (periodic x), a partial segment's two edge threads
// read (write) the one element beyond the segment directly.
//
// Addressing: the start of every row the tile touches (slot s, row y0 + dy
// of plane z + dz) is the same for every thread of the block; each thread
// adds one small 32-bit byte offset, shared by all 19 directions.
// BATCH: the instance of the tile and its parameters come from tables.
// Occupancy floor: 2-byte stores with 4 cells per thread sit near the
// register count of 3 wavefronts per SIMD, and the allocator sometimes lands
// just above it; hold it to 3.  The MRT odd step does not fit in that
// count: held to 3 it spills, and it ran 30 % faster at 2 without spills.
template <typename S, int V, bool ODD, bool MRT>
constexpr int min_waves() { return (sizeof(typename S::T) == 2 && V == 4 && !(ODD && MRT)) ? 3 : 1; }

// WHOLE: every block holds exactly one whole row, nx / V threads (the odd
// step's exchange then never needs a halo or a partial store, and that code
// is left out; the row is uniform over the block).
template <typename S, int V, bool ODD, int BCT, bool STATS, bool MRT, bool WHOLE>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(min_waves<S, V, ODD, MRT>()))) void k_step(StepArgs p0, const StepArgs* __restrict__ table,
                                                    const int* __restrict__ tile_inst, int ntiles_all)
{
    constexpr bool BATCH = (BCT == kBCRuntime);
    using T = typename S::T;
    using R = typename S::R;
    using Ln = Lane<S, V>;
    extern __shared__ u32x2 xbuf[];  // odd step: [kNX][blockDim.x]

    int tile;
    StepArgs p;
    if constexpr (BATCH) {
        const int gt = tile_of_block(blockIdx.x, ntiles_all, p0.xcd_remap);
        p = table[tile_inst[gt]];
        tile = gt - p.tile_begin;
    } else {
        p = p0;
        tile = tile_of_block(blockIdx.x, p.ntiles, p.xcd_remap);
    }
    tile = spread_tile(tile, p);
    const bool spec = BATCH ? (p.bc != kBB) : (BCT != kBB);
    const bool wfb = BATCH ? (p.bc == kWFB) : (BCT == kWFB);
    constexpr bool NODE = (BCT == kBCNode);          // wall nodes instead of halfway walls
    constexpr bool MAYBE_WFB = BATCH || BCT == kWFB;
    constexpr bool MAYBE_SPEC = BATCH || (BCT != kBB && !NODE);
    constexpr int cur = ODD ? 1 : 0, prev = 1 - cur; // wall-node rings written / read by this kernel
    // One cell per thread in row segments: the odd step's x-shifts are plain
    // address offsets (every load and store of a wavefront still covers
    // consecutive elements; the AA rule that a cell reads exactly the slots it
    // writes makes this race-free without an exchange or a barrier), which
    // also removes the segment halos.  Whole-row blocks and groups of V > 1
    // cells shift through LDS, so that every access stays aligned (measured on
    // MI355X, 2,048-cell rows in 256-cell segments: FP64 odd step 57.0 ->
    // 52.7 ms, FP32 with one cell per thread 26.3 ms against 28.7 ms with two
    // cells and the exchange).
    constexpr bool DIRECT = ODD && (V == 1) && !WHOLE;

    const long long N = p.n;
    const int t = (int)threadIdx.x;
    const int nthr = (int)blockDim.x;
    // tile -> (x segment, row group yt, z), numbered in memory order: x
    // segment, row group within its brick, z, brick
    const int rest = fdiv(tile, p.fd_ntx);
    const int xt = tile - rest * p.ntx;
    const int yb = fdiv(rest, p.fd_brick_tiles);
    const int rem = rest - yb * p.bgroups * p.nz;
    const bool last_brick = (yb == p.nbricks - 1);
    const int bgk = last_brick ? p.bg_last : p.bgroups;          // row groups of this brick
    const int z = last_brick ? fdiv(rem, p.fd_bg_last) : fdiv(rem, p.fd_bgroups);
    const int yt = yb * p.bgroups + (rem - z * bgk);
    // WHOLE: one whole row per block, so the row (y, the wall flags, the
    // row factors) is the same for every thread and stays in scalar registers
    const bool whole = WHOLE || (p.ntx == 1);
    const int tpr = whole ? p.nx / V : nthr;        // threads per row segment
    const int r = WHOLE ? 0 : fdiv(t, p.fd_tpr), tr = t - r * tpr;
    const int y = yt * p.rpb + r;
    const int seg0 = xt * nthr * V;                  // first cell of the segment
    const int nact = whole ? tpr : min(nthr, (p.nx - seg0) / V);
    RowLanes L;
    L.nx = p.nx;
    L.x0 = seg0 + tr * V;
    L.active = (r < p.rpb) && (y < p.ny) && (tr < nact);
    const bool bot = (y == 0), top = (y == p.ny - 1);
    const int lane = t & 63;
    const int tb = t - tr;                          // first thread of this row segment

    const int zm = (z == 0) ? p.nz - 1 : z - 1;
    const int zp = (z == p.nz - 1) ? 0 : z + 1;
    // The rows of a tile are consecutive in memory: a single row (bricked
    // layout) or rpb rows of one plane (plain layout).  Row (slot s, y + dy,
    // z + dz) starts at base(s, dy, dz) + row_off, where base is that of the
    // tile's first row y0 (uniform over the block) and row_off = (y - y0) nx
    // is the thread's part; neighbouring rows y0 + dy stay in the brick
    // except at its edges, where row_index steps to the next brick.
    const int y0 = yt * p.rpb;
    const int yi0 = y0 - yb * p.brick;                        // row of y0 within its brick
    const int bk = min(p.brick, p.ny - yb * p.brick);         // rows of this brick
    const bool plain = (p.brick >= p.ny);
    // memory row of (y0 + dy, zz): row_index without divisions, as selects
    // (evaluated once, outside any divergent branch, so it stays scalar)
    const int bkn = min(p.brick, p.ny - (yb + 1) * p.brick);  // rows of the next brick
    auto row_of = [&](int dy, int zz) -> long long {
        const int yi = yi0 + dy;
        const long long in_brick = (long long)yb * p.brick * p.nz + (long long)zz * bk + yi;
        const long long prev = ((long long)(yb - 1) * p.nz + zz) * p.brick + (p.brick - 1);
        const long long next = (long long)(yb + 1) * p.brick * p.nz + (long long)zz * bkn;
        const long long bricked = yi < 0 ? prev : (yi >= bk ? next : in_brick);
        return plain ? (long long)zz * p.ny + (y0 + dy) : bricked;
    };
    long long row_nx[3][3];  // [dy + 1][dz + 1]: element offset of the row within a slot
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz)
            row_nx[dy + 1][dz + 1] = row_of(dy, dz < 0 ? zm : (dz > 0 ? zp : z)) * p.nx;
    auto base = [&](int s, int dy, int dz) -> char* {
        return (char*)p.h + ((long long)s * N + row_nx[dy + 1][dz + 1]) * (long long)sizeof(T);
    };
    const unsigned row_off = (unsigned)(p.nx * (y - y0)) * (unsigned)sizeof(T);
    const unsigned lane_off = row_off + (unsigned)L.x0 * (unsigned)sizeof(T);
    auto at = [&](char* b, unsigned off) -> T* { return (T*)(b + off); };
    auto ld = [&](char* b) -> u32x2 { return Ln::template load<true>(at(b, lane_off)); };
    auto st = [&](char* b, u32x2 v) { Ln::template store<true>(at(b, lane_off), v); };
    // byte offset of element x of this thread's row
    auto xoff = [&](unsigned x) -> unsigned { return row_off + x * (unsigned)sizeof(T); };

    // a1/a2: gather.  Odd: pull from neighbours with wall reflections; even: own slots.
    u32x2 w[kQ];
    if (L.active) {
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            constexpr int ey = kEy[a], ez = kEz[a];
            if constexpr (NODE) {
                if ((ey == 1 && bot) || (ey == -1 && top)) {
                    // from the wall node at x - e_a: what it sent on the previous step
                    const int zz = ez > 0 ? zm : (ez < 0 ? zp : z);
                    w[a] = ring_load<S, V>(ring_row<S>(p, 2 + prev, top ? 1 : 0, node_k<a>(top), zz), L.x0, -kEx[a],
                                           p.nx);
                    return;
                }
            }
            if constexpr (ODD) {
                const bool from_wall = (ey == 1 && bot) || (ey == -1 && top);
                // one cell per thread: the x-shifted source element is loaded directly,
                // through the cache (the line a wavefront shares with its neighbour is then
                // fetched once; non-temporal shifted loads ran the odd step 5 % slower)
                constexpr bool SH = DIRECT && kEx[a] != 0;
                const unsigned soff = SH ? xoff(L.wrapx(L.x0 - kEx[a])) : lane_off;
                if (from_wall) {
                    if (MAYBE_SPEC && spec && is_tangential(a))
                        w[a] = Ln::template load<!SH>(at(base(opp(mirror_y(a)), 0, -ez), soff));
                    else w[a] = ld(base(a, 0, 0));
                } else {
                    w[a] = Ln::template load<!SH>(at(base(opp(a), -ey, -ez), soff));
                }
            } else {
                w[a] = ld(base(a, 0, 0));
            }
        });
    } else {
        for_each_dir([&](auto A) { w[decltype(A)::value] = u32x2{0u, 0u}; });
    }
    if constexpr (ODD && !DIRECT) {
        // the x-shifted groups hold cells x0 .. x0 + V - 1 of the source row; shift by -e_x
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            if constexpr (kEx[a] != 0) xbuf[xslot(a) * nthr + t] = w[a];
        });
        __syncthreads();
        if (L.active) {
            for_each_dir([&](auto A) {
                constexpr int a = decltype(A)::value;
                constexpr int ex = kEx[a], ey = kEy[a], ez = kEz[a];
                if constexpr (ex != 0) {
                    const bool from_wall = (ey == 1 && bot) || (ey == -1 && top);
                    const bool shifted = !from_wall || (MAYBE_SPEC && spec && is_tangential(a));
                    if (shifted) {
                        const u32x2* xb = xbuf + xslot(a) * nthr;
                        if constexpr (ex == 1) {  // needs the element at x0 - 1
                            u32x2 nb;
                            if (tr > 0) nb = xb[t - 1];
                            else if (whole) nb = xb[tb + nact - 1];
                            else nb = halo_as_last<S, V>(at(from_wall ? base(opp(mirror_y(a)), 0, -ez)
                                                                      : base(opp(a), -ey, -ez),
                                                            xoff(L.wrapx(L.x0 - 1))));
                            w[a] = join_left<S, V>(w[a], nb);
                        } else {                  // needs the element at x0 + V
                            u32x2 nb;
                            if (tr < nact - 1) nb = xb[t + 1];
                            else if (whole) nb = xb[tb];
                            else nb = halo_as_first<S, V>(at(from_wall ? base(opp(mirror_y(a)), 0, -ez)
                                                                       : base(opp(a), -ey, -ez),
                                                             xoff(L.wrapx(L.x0 + V))));
                            w[a] = join_right<S, V>(w[a], nb);
                        }
                    }
                }
            });
        }
    }

    // wall nodes: the collision of the populations that arrived there, with the
    // stress from the first layer's record of the previous step (mode 1); in
    // mode 2 it follows the record of this step, below
    if constexpr (NODE) {
        if (L.active && (bot || top) && p.wall_nodes != 2) node_collide<S, V>(p, top, z, L.x0, prev, cur);
    }

    double sm[7] = {0, 0, 0, 0, 0, 0, 0};
    int iters = 0;
    bool bad = false, newton_fail = false;
    double nrho[V], nux[V], nuz[V];   // wall nodes: the first layer's moments for the next wall-node collision
    // a3-a6 (the same steps as collide_group, written out here: the register
    // allocation of this kernel came out tighter this way)
    constexpr bool PAIRS = (sizeof(T) == 2) && (V >= 2);
    const bool wall_wfb = MAYBE_WFB && wfb && (bot || top) && L.active;
    MrtRates<R> mr;
    if constexpr (MRT) {
#pragma unroll
        for (int i = 0; i < 5; ++i) mr.s[i] = (R)p.mrt_s[i];
    }
    R whx[V], whz[V];
    if constexpr (MAYBE_WFB) {
        if (wall_wfb) wall_group<S, V>(w, p, whx, whz, iters, newton_fail);
    }
    auto cell = [&](int k, R (&f)[kQ]) {
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            f[a] = Ln::get(w[a], k);
        });
        if constexpr (MAYBE_WFB) {
            if (wall_wfb) wfb_apply<R>(f, top, whx[k], whz[k]);
        }
        // Smagorinsky factor of this row (van Driest damping)
        const R cs2 = (R)((p.cs2_row && L.active) ? p.cs2_row[y] : p.cs2_18);
        const Moments<R> m = collide<R, MRT>(f, (R)p.tau0, cs2, (R)p.fx, &mr);
        bad = bad || !(m.rho > R(0)) || !(m.rho < R(INFINITY));
        if constexpr (NODE) {
            nrho[k] = (double)m.rho;
            nux[k] = (double)m.ux;
            nuz[k] = (double)m.uz;
        }
        if constexpr (STATS) {
            const double ux = (double)m.ux, uy = (double)m.uy, uz = (double)m.uz;
            sm[0] += ux; sm[1] += uy; sm[2] += uz;
            sm[3] += ux * ux; sm[4] += uy * uy; sm[5] += uz * uz; sm[6] += ux * uy;
        }
    };
    if constexpr (PAIRS) {
#pragma unroll
        for (int k = 0; k < V; k += 2) {
            R f0[kQ], f1[kQ];
            cell(k, f0);
            cell(k + 1, f1);
            for_each_dir([&](auto A) {
                constexpr int a = decltype(A)::value;
                Ln::set_pair(w[a], k, f0[a], f1[a]);
            });
        }
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            R f[kQ];
            cell(k, f);
            for_each_dir([&](auto A) {
                constexpr int a = decltype(A)::value;
                Ln::set(w[a], k, f[a]);
            });
        }
    }
    if constexpr (NODE) {
        if (L.active && (bot || top)) {
            int it = 0;
            bool fl = false;
            node_record<V>(p, top, z, L.x0, nrho, nux, nuz, it, fl);
            iters = max(iters, it);
            newton_fail = newton_fail || fl;
            // the record of a node's column is this thread's own, and the arrivals
            // it collides came in the previous step (ring prev; this step's stores
            // fill ring cur)
            if (p.wall_nodes == 2) node_collide<S, V>(p, top, z, L.x0, prev, cur);
        }
    }
    if (L.active && (bad || newton_fail)) {
        atomicOr(&p.flags->status, (bad ? 1 : 0) | (newton_fail ? 2 : 0));
        atomicMin(&p.flags->first_bad, (unsigned long long)p.flags->cnt[ODD ? 1 : 0]);
    }

    // a7: store.  Odd: push to neighbours with wall reflections; even: own opposite slots.
    if constexpr (ODD) {
        if constexpr (!DIRECT) {
            __syncthreads();  // every thread is done reading the exchange buffer
            for_each_dir([&](auto A) {
                constexpr int a = decltype(A)::value;
                if constexpr (kEx[a] != 0) xbuf[xslot(a) * nthr + t] = w[a];
            });
            __syncthreads();
        }
        if (L.active) {
            for_each_dir([&](auto A) {
                constexpr int a = decltype(A)::value;
                constexpr int ex = kEx[a], ey = kEy[a], ez = kEz[a];
                const bool to_wall = (ey == -1 && bot) || (ey == 1 && top);
                if constexpr (NODE) {
                    if (to_wall) {   // towards the wall node at x + e_a
                        const int zz = ez > 0 ? zp : (ez < 0 ? zm : z);
                        ring_store<S, V>(ring_row<S>(p, cur, top ? 1 : 0, node_k<opp(a)>(top), zz), L.x0, ex, p.nx, w[a]);
                        return;
                    }
                }
                const bool mirrored = to_wall && MAYBE_SPEC && spec && is_tangential(a);
                if (to_wall && !mirrored) {
                    st(base(opp(a), 0, 0), w[a]);  // bounce-back into the cell's own slot
                } else if constexpr (ex == 0) {
                    st(mirrored ? base(mirror_y(a), 0, ez) : base(a, ey, ez), w[a]);
                } else if constexpr (DIRECT) {   // cell x goes to x + e_x (cached: lines shared with the neighbour)
                    char* dst = mirrored ? base(mirror_y(a), 0, ez) : base(a, ey, ez);
                    Ln::template store<false>(at(dst, xoff(L.wrapx(L.x0 + ex))), w[a]);
                } else {
                    char* dst = mirrored ? base(mirror_y(a), 0, ez) : base(a, ey, ez);
                    const u32x2* xb = xbuf + xslot(a) * nthr;
                    if constexpr (ex == 1) {  // cell x goes to x + 1: the group at x0 starts with x0 - 1's value
                        if (tr > 0 || whole) {
                            st(dst, join_left<S, V>(w[a], xb[tr > 0 ? t - 1 : tb + nact - 1]));
                        } else {
                            if constexpr (V > 1) Ln::store_tail(at(dst, lane_off), Ln::shift_in_left(w[a], 0u));
                        }
                        if (!whole && tr == nact - 1) {
                            if constexpr (V == 1) Ln::template store<false>(at(dst, xoff(L.wrapx(L.x0 + 1))), w[a]);
                            else Ln::store_elem(at(dst, xoff(L.wrapx(L.x0 + V))), Ln::last(w[a]));
                        }
                    } else {                  // cell x goes to x - 1: the group at x0 ends with x0 + V's value
                        if (tr < nact - 1 || whole) {
                            st(dst, join_right<S, V>(w[a], xb[tr < nact - 1 ? t + 1 : tb]));
                        } else {
                            if constexpr (V > 1) Ln::store_head(at(dst, lane_off), Ln::shift_in_right(w[a], 0u));
                        }
                        if (!whole && tr == 0) {
                            if constexpr (V == 1) Ln::template store<false>(at(dst, xoff(L.wrapx(L.x0 - 1))), w[a]);
                            else Ln::store_elem(at(dst, xoff(L.wrapx(L.x0 - 1))), Ln::first(w[a]));
                        }
                    }
                }
            });
        }
    } else {
        if (L.active) {
            for_each_dir([&](auto A) {
                constexpr int a = decltype(A)::value;
                if constexpr (NODE) {
                    constexpr int ey = kEy[a], ez = kEz[a];
                    if ((ey == -1 && bot) || (ey == 1 && top)) {   // towards the wall node at x + e_a
                        const int zz = ez > 0 ? zp : (ez < 0 ? zm : z);
                        ring_store<S, V>(ring_row<S>(p, cur, top ? 1 : 0, node_k<opp(a)>(top), zz), L.x0, kEx[a],
                                         p.nx, w[a]);
                        return;
                    }
                }
                st(base(opp(a), 0, 0), w[a]);
            });
        }
    }

    if constexpr (MAYBE_WFB || NODE) {
        const int mx = wave_max(L.active ? iters : 0);
        if (lane == 0 && mx > 0) atomicMax(&p.flags->max_newton_iters, mx);
    }
    // a8: plane statistics of the sampled velocity: FP64 sums per row segment,
    // threads of a row summed in a fixed order (sampled steps only)
    if constexpr (STATS) {
        __shared__ double red[7][kMaxBlock];
#pragma unroll
        for (int k = 0; k < 7; ++k) red[k][t] = L.active ? sm[k] : 0.0;
        __syncthreads();
        for (int idx = t; idx < 7 * p.rpb; idx += nthr) {
            const int rr = idx / 7, k = idx - rr * 7;
            const int yy = yt * p.rpb + rr;
            if (yy < p.ny) {
                double s = 0.0;
                for (int q = 0; q < tpr; ++q) s += red[k][rr * tpr + q];
                p.partials[((long long)xt + (long long)p.ntx * ((long long)yy + (long long)p.ny * z)) * 7 + k] = s;
            }
        }
    }
    if (tile == 0 && t == 0) p.flags->cnt[ODD ? 0 : 1] = p.flags->cnt[ODD ? 1 : 0] + 1;
}

// Edge elements of a group for the odd step by rows: one element's bits
// (V >= 2) or, for one-element groups, the group itself.
template <typename S, int V>
struct Edge {
    using Ln = Lane<S, V>;
    using E = std::conditional_t<V == 1, u32x2, unsigned int>;
    __device__ __forceinline__ static E last(u32x2 g)
    {
        if constexpr (V == 1) return g;
        else return Ln::last(g);
    }
    __device__ __forceinline__ static E first(u32x2 g)
    {
        if constexpr (V == 1) return g;
        else return Ln::first(g);
    }
    // [e, g0 .. g(V-2)] and [g1 .. g(V-1), e]
    __device__ __forceinline__ static u32x2 join_left(u32x2 g, E e)
    {
        if constexpr (V == 1) return e;
        else return Ln::shift_in_left(g, e);
    }
    __device__ __forceinline__ static u32x2 join_right(u32x2 g, E e)
    {
        if constexpr (V == 1) return e;
        else return Ln::shift_in_right(g, e);
    }
    __device__ __forceinline__ static E up(E e)  // lane i gets lane i - 1's value (lane 0 its own)
    {
        if constexpr (V == 1) return u32x2{(unsigned)__shfl_up((int)e.x, 1, 64), (unsigned)__shfl_up((int)e.y, 1, 64)};
        else return (unsigned)__shfl_up((int)e, 1, 64);
    }
    __device__ __forceinline__ static E down(E e)  // lane i gets lane i + 1's value (lane 63 its own)
    {
        if constexpr (V == 1)
            return u32x2{(unsigned)__shfl_down((int)e.x, 1, 64), (unsigned)__shfl_down((int)e.y, 1, 64)};
        else return (unsigned)__shfl_down((int)e, 1, 64);
    }
    __device__ __forceinline__ static E lane_value(E e, int l)  // lane l's value, wave-uniform
    {
        if constexpr (V == 1)
            return u32x2{(unsigned)__builtin_amdgcn_readlane((int)e.x, l), (unsigned)__builtin_amdgcn_readlane((int)e.y, l)};
        else return (unsigned)__builtin_amdgcn_readlane((int)e, l);
    }
    __device__ __forceinline__ static u32x2 lane_group(u32x2 g, int l)
    {
        return u32x2{(unsigned)__builtin_amdgcn_readlane((int)g.x, l), (unsigned)__builtin_amdgcn_readlane((int)g.y, l)};
    }
    __device__ __forceinline__ static E uniform(E e)  // a value every lane holds alike, as a scalar
    {
        if constexpr (V == 1)
            return u32x2{(unsigned)__builtin_amdgcn_readfirstlane((int)e.x), (unsigned)__builtin_amdgcn_readfirstlane((int)e.y)};
        else return (unsigned)__builtin_amdgcn_readfirstlane((int)e);
    }
    // the element at p (every lane loads the same address)
    __device__ __forceinline__ static E load_at(const typename S::T* p)
    {
        if constexpr (V == 1) return Ln::template load<false>(p);
        else return Ln::load_elem(p);
    }
};

// The odd step by rows, for rows of whole 64-lane segments.  Each wavefront
// owns one row (a block holds blockDim.x / 64 consecutive rows in memory
// order) and walks it in nseg segments of 64 V cells.  The x-shift of the
// streamwise directions moves one element across lanes by a shuffle; across
// segments, and around the periodic row, the edge elements are carried in
// scalar registers:
//   gather, e_x = +1: lane 0 takes the previous segment's last element (for
//     the first segment: the row's last element, loaded at the start);
//   gather, e_x = -1: lane 63 takes the next segment's first element, loaded
//     with the segment (for the last segment: the row's first element, kept
//     from the first segment);
//   store, e_x = +1: the first segment's first group waits for the row's last
//     post-collision element; the row's first 128-byte line is held in LDS and
//     written whole after the walk;
//   store, e_x = -1: each segment's last group waits for the next segment's
//     first post-collision element (the row's first one for the last
//     segment); the segment's last 128-byte line is held in LDS and written
//     whole one segment later.
// So every line is written by one store of one wavefront: no partial lines
// reach the memory.  Every element a cell reads is read before any cell
// writes it: an AA cell reads exactly the slots it writes, and carried
// elements are taken from the loads of their own segment.  No barrier: the
// lines held in LDS are only ever read by the wavefront that wrote them.
template <typename S, int V, int BCT, bool STATS, bool MRT>
__global__ __launch_bounds__(kMaxBlock) void k_odd_rows(StepArgs p0, const StepArgs* __restrict__ table,
                                                        const int* __restrict__ tile_inst, int ntiles_all)
{
    constexpr bool BATCH = (BCT == kBCRuntime);
    using T = typename S::T;
    using Ln = Lane<S, V>;
    using Ed = Edge<S, V>;
    using E = typename Ed::E;
    constexpr bool MAYBE_WFB = BATCH || BCT == kWFB;
    constexpr bool MAYBE_SPEC = BATCH || BCT != kBB;

    int tile;
    StepArgs p;
    if constexpr (BATCH) {
        const int gt = tile_of_block(blockIdx.x, ntiles_all, p0.xcd_remap);
        p = table[tile_inst[gt]];
        tile = gt - p.tile_begin;
    } else {
        p = p0;
        tile = tile_of_block(blockIdx.x, p.ntiles, p.xcd_remap);
    }
    tile = spread_tile(tile, p);
    const bool spec = BATCH ? (p.bc != kBB) : (BCT != kBB);
    const bool wfb = BATCH ? (p.bc == kWFB) : (BCT == kWFB);
    if (tile == 0 && threadIdx.x == 0) p.flags->cnt[0] = p.flags->cnt[1] + 1;

    const int lane = (int)threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int row = tile * ((int)blockDim.x >> 6) + wave;   // memory-order row of this wavefront
    if (row >= p.ny * p.nz) return;
    // memory row -> (brick, z, row in brick) -> (y, z)
    const int yb = fdiv(row, p.fd_brick_tiles);
    const int rem = row - yb * p.bgroups * p.nz;
    const bool last_brick = (yb == p.nbricks - 1);
    const int bk = last_brick ? p.bg_last : p.bgroups;         // rows of this brick
    const int z = last_brick ? fdiv(rem, p.fd_bg_last) : fdiv(rem, p.fd_bgroups);
    const int yi0 = rem - z * bk;
    const int y = yb * p.brick + yi0;
    const bool bot = (y == 0), top = (y == p.ny - 1);
    const typename S::R cs2 = (typename S::R)(p.cs2_row ? p.cs2_row[y] : p.cs2_18);  // van Driest damping
    const int zm = (z == 0) ? p.nz - 1 : z - 1;
    const int zp = (z == p.nz - 1) ? 0 : z + 1;
    const bool plain = (p.brick >= p.ny);
    const int bkn = min(p.brick, p.ny - (yb + 1) * p.brick);
    auto row_of = [&](int dy, int zz) -> long long {
        const int yi = yi0 + dy;
        const long long in_brick = (long long)yb * p.brick * p.nz + (long long)zz * bk + yi;
        const long long prev = ((long long)(yb - 1) * p.nz + zz) * p.brick + (p.brick - 1);
        const long long next = (long long)(yb + 1) * p.brick * p.nz + (long long)zz * bkn;
        const long long bricked = yi < 0 ? prev : (yi >= bk ? next : in_brick);
        return plain ? (long long)zz * p.ny + (y + dy) : bricked;
    };
    long long row_nx[3][3];
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz)
            row_nx[dy + 1][dz + 1] = row_of(dy, dz < 0 ? zm : (dz > 0 ? zp : z)) * p.nx;
    const long long N = p.n;
    // The row starts are recomputed in every segment from hbits, which the
    // empty asm statement makes opaque to the compiler: kept live across the
    // walk, 38 of them would not fit in scalar registers.
    typedef __attribute__((address_space(1))) char gchar;   // global memory, so that loads stay global
    unsigned long long hbits = (unsigned long long)p.h;
    auto base = [&](int s, int dy, int dz) -> char* {
        gchar* g = (gchar*)hbits;
        return (char*)(g + ((long long)s * N + row_nx[dy + 1][dz + 1]) * (long long)sizeof(T));
    };
    auto at = [&](char* b, unsigned off) -> T* { return (T*)(b + off); };
    // the source row of direction a (its x-shift applies unless it is bounced back unshifted)
    auto src_of = [&](auto A) -> char* {
        constexpr int a = decltype(A)::value;
        constexpr int ey = kEy[a], ez = kEz[a];
        const bool from_wall = (ey == 1 && bot) || (ey == -1 && top);
        if (from_wall) return (MAYBE_SPEC && spec && is_tangential(a)) ? base(opp(mirror_y(a)), 0, -ez) : base(a, 0, 0);
        return base(opp(a), -ey, -ez);
    };
    auto shifted_in = [&](auto A) -> bool {
        constexpr int a = decltype(A)::value;
        constexpr int ey = kEy[a];
        const bool from_wall = (ey == 1 && bot) || (ey == -1 && top);
        return kEx[a] != 0 && (!from_wall || (MAYBE_SPEC && spec && is_tangential(a)));
    };
    // the destination row of direction a and whether its x-shift applies
    auto dst_of = [&](auto A) -> char* {
        constexpr int a = decltype(A)::value;
        constexpr int ey = kEy[a], ez = kEz[a];
        const bool to_wall = (ey == -1 && bot) || (ey == 1 && top);
        const bool mirrored = to_wall && MAYBE_SPEC && spec && is_tangential(a);
        if (to_wall && !mirrored) return base(opp(a), 0, 0);  // bounce-back into the cell's own slot
        return mirrored ? base(mirror_y(a), 0, ez) : base(a, ey, ez);
    };
    auto shifted_out = [&](auto A) -> bool {
        constexpr int a = decltype(A)::value;
        constexpr int ey = kEy[a];
        const bool to_wall = (ey == -1 && bot) || (ey == 1 && top);
        const bool mirrored = to_wall && MAYBE_SPEC && spec && is_tangential(a);
        return kEx[a] != 0 && (!to_wall || mirrored);
    };

    const int nseg = p.nseg;
    const unsigned sbytes = (unsigned)sizeof(T);
    E gcar[kNX], gwrap[kNX], scar[kNX], swrap[kNX];
    // lanes whose groups fill one 128-byte line
    constexpr int G = 128 / (V * (int)sizeof(T));
    static_assert(G >= 16 && G <= 64 && 128 % (V * (int)sizeof(T)) == 0, "groups of 2, 4 or 8 bytes");
    // lines held back per wavefront and shifted direction: e_x = +1, the row's
    // first line (lanes 0 .. G - 1 of the first segment, written after the
    // walk); e_x = -1, the current segment's last line (lanes 64 - G .. 63,
    // written by lanes 0 .. G - 1 of the next segment or after the walk).
    // A wavefront reads only what it wrote itself; the wave barriers keep the
    // compiler from moving these LDS accesses across each other.
    __shared__ u32x2 hold[kMaxBlock / 64][kNX][G];
    // the row's last element for the first segment's e_x = +1 gather
    for_each_dir([&](auto A) {
        constexpr int a = decltype(A)::value;
        if constexpr (kEx[a] == 1) {
            if (shifted_in(A)) gcar[xslot(a)] = Ed::uniform(Ed::load_at(at(src_of(A), (unsigned)(p.nx - 1) * sbytes)));
        }
    });

    double sm[7] = {0, 0, 0, 0, 0, 0, 0};
    int iters = 0;
    bool bad = false, newton_fail = false;
    for (int k = 0; k < nseg; ++k) {
        asm volatile("" : "+s"(hbits));
        const unsigned off = (unsigned)((k * 64 + lane) * V) * sbytes;
        const bool more = (k + 1 < nseg);
        // a1/a2: gather with wall reflections
        u32x2 w[kQ];
        E ahead[kNX] = {};
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            w[a] = Ln::template load<true>(at(src_of(A), off));
            if constexpr (kEx[a] == -1) {  // the next segment's first element (every lane loads it alike)
                if (more && shifted_in(A))
                    ahead[xslot(a)] = Ed::load_at(at(src_of(A), (unsigned)((k + 1) * 64 * V) * sbytes));
            }
        });
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            if constexpr (kEx[a] != 0) {
                if (shifted_in(A)) {
                    constexpr int j = xslot(a);
                    if constexpr (kEx[a] == 1) {      // needs the element at x0 - 1
                        const E mine = Ed::last(w[a]);
                        E nb = Ed::up(mine);
                        if (lane == 0) nb = gcar[j];
                        gcar[j] = Ed::lane_value(mine, 63);
                        w[a] = Ed::join_left(w[a], nb);
                    } else {                          // needs the element at x0 + V
                        const E mine = Ed::first(w[a]);
                        if (k == 0) gwrap[j] = Ed::lane_value(mine, 0);
                        E nb = Ed::down(mine);
                        if (lane == 63) nb = more ? Ed::uniform(ahead[j]) : gwrap[j];
                        w[a] = Ed::join_right(w[a], nb);
                    }
                }
            }
        });
        // a3-a6
        collide_group<S, V, MAYBE_WFB, STATS, MRT>(w, p, cs2, wfb && (bot || top), top, sm, iters, bad, newton_fail);
        // a7: store with wall reflections
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            char* dst = dst_of(A);
            if constexpr (kEx[a] == 0) {
                Ln::template store<true>(at(dst, off), w[a]);
            } else {
                if (!shifted_out(A)) {
                    Ln::template store<true>(at(dst, off), w[a]);
                } else {
                    constexpr int j = xslot(a);
                    if constexpr (kEx[a] == 1) {      // the group at x0 starts with x0 - 1's value
                        const E mine = Ed::last(w[a]);
                        E pv = Ed::up(mine);
                        if (lane == 0) pv = scar[j];
                        scar[j] = Ed::lane_value(mine, 63);
                        if (k == 0 && lane < G)       // the row's first line waits for the row's last element
                            hold[wave][j][lane] = (lane == 0) ? w[a] : Ed::join_left(w[a], pv);
                        else
                            Ln::template store<true>(at(dst, off), Ed::join_left(w[a], pv));
                    } else {                          // the group at x0 ends with x0 + V's value
                        const E mine = Ed::first(w[a]);
                        const E pv = Ed::down(mine);
                        const E first0 = Ed::lane_value(mine, 0);
                        if (k == 0) {
                            swrap[j] = first0;
                        } else if (lane < G) {        // the previous segment's last line, now complete
                            u32x2 g = hold[wave][j][lane];
                            if (lane == G - 1) g = Ed::join_right(g, first0);
                            Ln::template store<true>(at(dst, off - (unsigned)(G * V) * sbytes), g);
                        }
                        __builtin_amdgcn_wave_barrier();
                        if (lane >= 64 - G)           // this segment's last line waits for the next segment
                            hold[wave][j][lane - (64 - G)] = (lane == 63) ? w[a] : Ed::join_right(w[a], pv);
                        else
                            Ln::template store<true>(at(dst, off), Ed::join_right(w[a], pv));
                    }
                }
            }
        });
    }
    // the lines that waited for the other end of the periodic row
    __builtin_amdgcn_wave_barrier();
    if (lane < G) {
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            if constexpr (kEx[a] != 0) {
                if (shifted_out(A)) {
                    constexpr int j = xslot(a);
                    char* dst = dst_of(A);
                    u32x2 g = hold[wave][j][lane];
                    if constexpr (kEx[a] == 1) {
                        if (lane == 0) g = Ed::join_left(g, scar[j]);
                        Ln::template store<true>(at(dst, (unsigned)(lane * V) * sbytes), g);
                    } else {
                        if (lane == G - 1) g = Ed::join_right(g, swrap[j]);
                        Ln::template store<true>(at(dst, (unsigned)(p.nx - (G - lane) * V) * sbytes), g);
                    }
                }
            }
        });
    }
    if (bad || newton_fail) {
        atomicOr(&p.flags->status, (bad ? 1 : 0) | (newton_fail ? 2 : 0));
        atomicMin(&p.flags->first_bad, (unsigned long long)p.flags->cnt[1]);
    }
    if constexpr (MAYBE_WFB) {
        const int mx = wave_max(iters);
        if (lane == 0 && mx > 0) atomicMax(&p.flags->max_newton_iters, mx);
    }
    // a8: plane statistics: the row's sums (fixed-order wave reduction)
    if constexpr (STATS) {
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            const double v = wave_sum(sm[q]);
            if (lane == 0) p.partials[((long long)y + (long long)p.ny * z) * 7 + q] = v;
        }
    }
}

template <typename S, int V, bool MRT>
static hipError_t launch_odd_rows(int bc, const StepArgs& a, hipStream_t s)
{
    const dim3 grid((unsigned)a.ntiles), block((unsigned)a.tile_x);
#define LBM_ROWS(BCT)                                                                                          \
    do {                                                                                                       \
        if (a.partials)                                                                                        \
            hipLaunchKernelGGL((k_odd_rows<S, V, BCT, true, MRT>), grid, block, 0, s, a, nullptr, nullptr, 0); \
        else                                                                                                   \
            hipLaunchKernelGGL((k_odd_rows<S, V, BCT, false, MRT>), grid, block, 0, s, a, nullptr, nullptr, 0);\
    } while (0)
    if (bc == kBB) LBM_ROWS(kBB);
    else if (bc == kWFB) LBM_ROWS(kWFB);
    else LBM_ROWS(kFreeSlip);
#undef LBM_ROWS
    return hipGetLastError();
}

// Blocks of exactly one whole row: nx / V threads per block.
inline bool whole_row_blocks(const StepArgs& a) { return a.ntx == 1 && a.rpb == 1 && a.nx == a.vw * a.tile_x; }

template <typename S, int V, bool ODD, bool MRT>
static hipError_t launch_step_bc(int bc, const StepArgs& a, hipStream_t s)
{
    if constexpr (ODD)
        if (a.nseg > 0) {
            if (a.wall_nodes) return hipErrorInvalidValue;   // wall nodes run the block kernel
            return launch_odd_rows<S, V, MRT>(bc, a, s);
        }
    const dim3 grid((unsigned)a.ntiles), block((unsigned)a.tile_x);
    // the odd step's LDS exchange (one-cell row segments shift directly)
    const size_t lds_x = (size_t)kNX * a.tile_x * sizeof(u32x2);
#define LBM_STEP_W(BCT, W)                                                                                          \
    do {                                                                                                            \
        const size_t lds = (ODD && (V > 1 || W)) ? lds_x : 0;                                                       \
        if (a.partials)                                                                                             \
            hipLaunchKernelGGL((k_step<S, V, ODD, BCT, true, MRT, W>), grid, block, lds, s, a, nullptr, nullptr, 0);  \
        else                                                                                                        \
            hipLaunchKernelGGL((k_step<S, V, ODD, BCT, false, MRT, W>), grid, block, lds, s, a, nullptr, nullptr, 0); \
    } while (0)
    // blocks of one whole row run the kernel without segment code
#define LBM_STEP(BCT)                                         \
    do {                                                      \
        if (whole_row_blocks(a)) LBM_STEP_W(BCT, true);       \
        else LBM_STEP_W(BCT, false);                          \
    } while (0)
    if (a.wall_nodes) LBM_STEP(kBCNode);
    else if (bc == kBB) LBM_STEP(kBB);
    else if (bc == kWFB) LBM_STEP(kWFB);
    else LBM_STEP(kFreeSlip);
#undef LBM_STEP
#undef LBM_STEP_W
    return hipGetLastError();
}

template <typename S, int V, bool MRT>
static hipError_t launch_batch_v(bool odd, const StepArgs& a0, const StepArgs* table, const int* tile_inst, int ntiles,
                                 hipStream_t s)
{
    const dim3 grid((unsigned)ntiles), block((unsigned)a0.tile_x);
    const size_t lds = (odd && V > 1) ? (size_t)kNX * a0.tile_x * sizeof(u32x2) : 0;
    if (odd && a0.nseg > 0)
        hipLaunchKernelGGL((k_odd_rows<S, V, kBCRuntime, false, MRT>), grid, block, 0, s, a0, table, tile_inst, ntiles);
    else if (odd)
        hipLaunchKernelGGL((k_step<S, V, true, kBCRuntime, false, MRT, false>), grid, block, lds, s, a0, table,
                           tile_inst, ntiles);
    else
        hipLaunchKernelGGL((k_step<S, V, false, kBCRuntime, false, MRT, false>), grid, block, lds, s, a0, table,
                           tile_inst, ntiles);
    return hipGetLastError();
}

// Dispatch on the group width (cells per thread) the store allows.
template <typename S, typename F>
static hipError_t with_width(int vw, F&& f)
{
    constexpr int kB = (int)sizeof(typename S::T);
    if (vw == 1) return f(std::integral_constant<int, 1>{});
    if constexpr (kB <= 4)
        if (vw == 2) return f(std::integral_constant<int, 2>{});
    if constexpr (kB == 2)
        if (vw == 4) return f(std::integral_constant<int, 4>{});
    return hipErrorInvalidValue;
}

// The per-store entry points declared in lbm_internal.h; each step_*.hip
// file instantiates them for its store.
template <typename S>
hipError_t launch_step_store(bool odd, int bc, const StepArgs& a, hipStream_t s)
{
    return with_width<S>(a.vw, [&](auto Vc) {
        constexpr int V = decltype(Vc)::value;
        if (a.coll == kMRT)
            return odd ? launch_step_bc<S, V, true, true>(bc, a, s) : launch_step_bc<S, V, false, true>(bc, a, s);
        return odd ? launch_step_bc<S, V, true, false>(bc, a, s) : launch_step_bc<S, V, false, false>(bc, a, s);
    });
}

template <typename S>
hipError_t launch_batch_store(bool odd, const StepArgs& a0, const StepArgs* table, const int* tile_inst, int ntiles,
                              hipStream_t s)
{
    return with_width<S>(a0.vw, [&](auto Vc) {
        if (a0.coll == kMRT) return launch_batch_v<S, decltype(Vc)::value, true>(odd, a0, table, tile_inst, ntiles, s);
        return launch_batch_v<S, decltype(Vc)::value, false>(odd, a0, table, tile_inst, ntiles, s);
    });
}

}  // namespace lbmwf
