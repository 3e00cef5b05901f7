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

// Boundary of a launch: fixed at compile time for a single channel, read
// from the instance table for batched launches (instances differ).
constexpr int kBCRuntime = 3;

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
template <typename S, int V, bool ODD, int BCT, bool STATS>
__global__ __launch_bounds__(kMaxBlock) void k_step(StepArgs p0, const StepArgs* __restrict__ table,
                                                    const int* __restrict__ tile_inst, int ntiles_all)
{
    constexpr bool BATCH = (BCT == kBCRuntime);
    using T = typename S::T;
    using R = typename S::R;
    using Ln = Lane<S, V>;
    constexpr bool PAIRS = (sizeof(T) == 2) && (V >= 2);
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
    const bool spec = BATCH ? (p.bc != kBB) : (BCT != kBB);
    const bool wfb = BATCH ? (p.bc == kWFB) : (BCT == kWFB);
    constexpr bool MAYBE_WFB = BATCH || BCT == kWFB;
    constexpr bool MAYBE_SPEC = BATCH || BCT != kBB;

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
    const bool whole = (p.ntx == 1);
    const int tpr = whole ? p.nx / V : nthr;        // threads per row segment
    const int r = fdiv(t, p.fd_tpr), tr = t - r * tpr;
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
            if constexpr (ODD) {
                const bool from_wall = (ey == 1 && bot) || (ey == -1 && top);
                if (from_wall) {
                    if (MAYBE_SPEC && spec && is_tangential(a)) w[a] = ld(base(opp(mirror_y(a)), 0, -ez));
                    else w[a] = ld(base(a, 0, 0));
                } else {
                    w[a] = ld(base(opp(a), -ey, -ez));
                }
            } else {
                w[a] = ld(base(a, 0, 0));
            }
        });
    } else {
        for_each_dir([&](auto A) { w[decltype(A)::value] = u32x2{0u, 0u}; });
    }
    if constexpr (ODD) {
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

    double sm[7] = {0, 0, 0, 0, 0, 0, 0};
    int iters = 0;
    bool bad = false, newton_fail = false;
    // a3-a6 for cell k of the group: decode, wall function, collision
    auto cell = [&](int k, R (&f)[kQ]) {
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            f[a] = Ln::get(w[a], k);
        });
        // a3: wall-function bounce at wall-adjacent cells
        if constexpr (MAYBE_WFB) {
            if (wfb && (bot || top) && L.active) {
                int it = 0;
                bool fail = false;
                wfb_correct<R>(f, top, p.fx, p.y1, p.nu0, p.kappa, p.bconst, p.ekb, p.newton_tol, p.newton_maxit, it,
                               fail);
                iters = max(iters, it);
                newton_fail = newton_fail || fail;
            }
        }
        // a4-a6: moments, Smagorinsky, BGK + body force
        const Moments<R> m = collide<R>(f, (R)p.tau0, (R)p.cs2_18, (R)p.fx);
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
    if (L.active && (bad || newton_fail)) {
        atomicOr(&p.flags->status, (bad ? 1 : 0) | (newton_fail ? 2 : 0));
        atomicMin(&p.flags->first_bad, (unsigned long long)p.flags->cnt[ODD ? 1 : 0]);
    }

    // a7: store.  Odd: push to neighbours with wall reflections; even: own opposite slots.
    if constexpr (ODD) {
        __syncthreads();  // every thread is done reading the exchange buffer
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            if constexpr (kEx[a] != 0) xbuf[xslot(a) * nthr + t] = w[a];
        });
        __syncthreads();
        if (L.active) {
            for_each_dir([&](auto A) {
                constexpr int a = decltype(A)::value;
                constexpr int ex = kEx[a], ey = kEy[a], ez = kEz[a];
                const bool to_wall = (ey == -1 && bot) || (ey == 1 && top);
                const bool mirrored = to_wall && MAYBE_SPEC && spec && is_tangential(a);
                if (to_wall && !mirrored) {
                    st(base(opp(a), 0, 0), w[a]);  // bounce-back into the cell's own slot
                } else if constexpr (ex == 0) {
                    st(mirrored ? base(mirror_y(a), 0, ez) : base(a, ey, ez), w[a]);
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
                st(base(opp(a), 0, 0), w[a]);
            });
        }
    }

    if constexpr (MAYBE_WFB) {
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

template <typename S, int V, bool ODD>
static hipError_t launch_step_bc(int bc, const StepArgs& a, hipStream_t s)
{
    const dim3 grid((unsigned)a.ntiles), block((unsigned)a.tile_x);
    const size_t lds = ODD ? (size_t)kNX * a.tile_x * sizeof(u32x2) : 0;
#define LBM_STEP(BCT)                                                                                        \
    do {                                                                                                     \
        if (a.partials)                                                                                      \
            hipLaunchKernelGGL((k_step<S, V, ODD, BCT, true>), grid, block, lds, s, a, nullptr, nullptr, 0);  \
        else                                                                                                 \
            hipLaunchKernelGGL((k_step<S, V, ODD, BCT, false>), grid, block, lds, s, a, nullptr, nullptr, 0); \
    } while (0)
    if (bc == kBB) LBM_STEP(kBB);
    else if (bc == kWFB) LBM_STEP(kWFB);
    else LBM_STEP(kFreeSlip);
#undef LBM_STEP
    return hipGetLastError();
}

template <typename S, int V>
static hipError_t launch_batch_v(bool odd, const StepArgs& a0, const StepArgs* table, const int* tile_inst, int ntiles,
                                 hipStream_t s)
{
    const dim3 grid((unsigned)ntiles), block((unsigned)a0.tile_x);
    const size_t lds = odd ? (size_t)kNX * a0.tile_x * sizeof(u32x2) : 0;
    if (odd)
        hipLaunchKernelGGL((k_step<S, V, true, kBCRuntime, false>), grid, block, lds, s, a0, table, tile_inst, ntiles);
    else
        hipLaunchKernelGGL((k_step<S, V, false, kBCRuntime, false>), grid, block, lds, s, a0, table, tile_inst, ntiles);
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
        return odd ? launch_step_bc<S, V, true>(bc, a, s) : launch_step_bc<S, V, false>(bc, a, s);
    });
}

template <typename S>
hipError_t launch_batch_store(bool odd, const StepArgs& a0, const StepArgs* table, const int* tile_inst, int ntiles,
                              hipStream_t s)
{
    return with_width<S>(a0.vw, [&](auto Vc) {
        return launch_batch_v<S, decltype(Vc)::value>(odd, a0, table, tile_inst, ntiles, s);
    });
}

}  // namespace lbmwf
