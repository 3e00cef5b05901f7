// Device kernels of the channel library other than the time step (initial
// state, state transfer, observation, statistics reduction, re-reflection,
// probes), and the host-side launch geometry and dispatch of the step kernels
// (lbm_step.h).
//
// Method: Han, Ooka & Kikumoto, "A wall function approach in lattice
// Boltzmann method" (arXiv 2009.04352).
#include "lbm_device.h"

namespace lbmwf {

// Largest group width the store and the row length allow: 8-byte groups.
int step_vector_width(int store, int nx)
{
    int vw = 8 / store_bytes(store);
    while (vw > 1 && nx % vw != 0) vw /= 2;
    return vw;
}

bool step_vector_width_ok(int store, int nx, int vw)
{
    return vw >= 1 && vw * store_bytes(store) <= 8 && (vw & (vw - 1)) == 0 && nx % vw == 0;
}

// A bricked layout (brick < ny) needs single-row tiles: the rows of a tile
// must be consecutive in memory with the same neighbours.
bool brick_ok(int ny, int brick, int rpb)
{
    return brick >= 1 && brick <= ny && (rpb == 1 || brick == ny);
}

void step_geometry(int nx, int ny, int nz, int tile_x, int vw, int brick, StepArgs& a)
{
    a.tile_x = tile_x;
    a.vw = vw;
    const int tpr_full = nx / vw;
    if (tpr_full <= tile_x) {  // whole rows, several per block when they are short
        a.ntx = 1;
        a.rpb = tile_x / tpr_full;
    } else {
        a.ntx = (tpr_full + tile_x - 1) / tile_x;
        a.rpb = 1;
    }
    a.nyt = (ny + a.rpb - 1) / a.rpb;
    a.ntiles = a.ntx * a.nyt * nz;
    a.brick = brick;
    a.bgroups = (brick >= ny) ? a.nyt : brick / a.rpb;
    if (a.bgroups < 1) a.bgroups = 1;  // rejected by brick_ok; keeps the divisors positive
    a.nbricks = (a.nyt + a.bgroups - 1) / a.bgroups;
    a.bg_last = a.nyt - (a.nbricks - 1) * a.bgroups;
    a.fd_ntx = make_fastdiv(a.ntx);
    a.fd_brick_tiles = make_fastdiv(a.bgroups * nz);
    a.fd_bgroups = make_fastdiv(a.bgroups);
    a.fd_bg_last = make_fastdiv(a.bg_last);
    a.fd_tpr = make_fastdiv(a.ntx == 1 ? tpr_full : tile_x);
    a.nseg = 0;
    set_spread(a, 0);
}

// The odd step by rows needs rows of whole 64-lane segments.
bool rows_ok(int nx, int vw) { return nx % (64 * vw) == 0; }

// Geometry of the odd step by rows: a tile is tile_x / 64 consecutive rows in
// memory order, one per wavefront; the decomposition of a memory row into
// (brick, z, row in brick) uses the fields of single-row tiles.
void step_geometry_rows(int nx, int ny, int nz, int tile_x, int vw, int brick, StepArgs& a)
{
    step_geometry(nx, ny, nz, tile_x, vw, brick, a);   // for vw and the common fields
    a.ntx = 1;
    a.rpb = 1;
    a.nyt = ny;
    a.bgroups = brick >= ny ? ny : brick;
    a.nbricks = (ny + a.bgroups - 1) / a.bgroups;
    a.bg_last = ny - (a.nbricks - 1) * a.bgroups;
    a.fd_ntx = make_fastdiv(1);
    a.fd_brick_tiles = make_fastdiv(a.bgroups * nz);
    a.fd_bgroups = make_fastdiv(a.bgroups);
    a.fd_bg_last = make_fastdiv(a.bg_last);
    a.fd_tpr = make_fastdiv(tile_x);
    const int waves = tile_x / 64;
    a.ntiles = (int)(((long long)ny * nz + waves - 1) / waves);
    a.nseg = nx / (64 * vw);
    set_spread(a, 0);
}

// Launch order that spreads the bricks over time: chunks of 2^log2 tiles
// cycle through the bricks (round q of chunks takes chunk q of every brick),
// so the wall rows, which live in the first and last brick and cost more
// than the others (the wall-function Newton solve), are mixed into the whole
// launch instead of its first and last 1/nbricks.  log2 <= 0, a single
// brick, a short last brick or bricks that are not a whole number of chunks
// keep the memory order.  Chunks smaller than a round of XCD chunks (8 of
// 2^kXcdChunkLog2 tiles, one per XCD) would give each XCD the same few
// bricks when the brick count is even; rotating round q's bricks by q
// avoids that.
void set_spread(StepArgs& a, int log2)
{
    const long long brick_tiles = (a.nseg > 0) ? (long long)a.bgroups * a.nz : (long long)a.ntx * a.bgroups * a.nz;
    const int waves = (a.nseg > 0) ? a.tile_x / 64 : 1;   // rows per tile of the odd step by rows
    a.tiles_per_brick = (int)(brick_tiles / waves);
    a.fd_nbricks = make_fastdiv(a.nbricks);
    const bool ok = log2 > 0 && log2 < 30 && a.nbricks > 1 && a.bg_last == a.bgroups && brick_tiles % waves == 0 &&
                    a.tiles_per_brick % (1 << log2) == 0;
    a.spread = ok ? log2 : -1;
    a.spread_rot = (a.nbricks % 2 == 0 && log2 < kXcdChunkLog2 + 3) ? 1 : 0;
}

static bool step_args_ok(int store, const StepArgs& a)
{
    if (a.tile_x < 64 || a.tile_x > kMaxBlock || (a.tile_x & 63) || a.ntiles < 1) return false;
    if (a.wall_nodes && (!a.wn || !a.wn_rec || a.nseg > 0)) return false;
    if (!step_vector_width_ok(store, a.nx, a.vw)) return false;
    // the thread part of an address is (row in tile * nx + x) * bytes < 32 bits
    if ((long long)a.nx * a.ny * store_bytes(store) > 0xffffffffll) return false;
    StepArgs g = a;
    if (a.nseg > 0) {
        if (!rows_ok(a.nx, a.vw)) return false;
        step_geometry_rows(a.nx, a.ny, a.nz, a.tile_x, a.vw, a.brick, g);
        if (a.brick < 1 || a.brick > a.ny || g.nseg != a.nseg) return false;
    } else {
        step_geometry(a.nx, a.ny, a.nz, a.tile_x, a.vw, a.brick, g);
        if (!brick_ok(a.ny, a.brick, g.rpb)) return false;
    }
    set_spread(g, a.spread);
    // the decomposition must be the one step_geometry derives (the batched
    // launch reads it from the device table)
    auto same = [](const FastDiv& x, const FastDiv& y) { return x.m == y.m && x.s == y.s; };
    return g.ntx == a.ntx && g.rpb == a.rpb && g.nyt == a.nyt && g.ntiles == a.ntiles && g.bgroups == a.bgroups &&
           g.nbricks == a.nbricks && g.bg_last == a.bg_last && same(g.fd_ntx, a.fd_ntx) &&
           same(g.fd_brick_tiles, a.fd_brick_tiles) && same(g.fd_bgroups, a.fd_bgroups) &&
           same(g.fd_bg_last, a.fd_bg_last) && same(g.fd_tpr, a.fd_tpr) && g.spread == a.spread &&
           (a.spread < 0 || (a.spread_rot == g.spread_rot && a.tiles_per_brick == g.tiles_per_brick &&
                             same(g.fd_nbricks, a.fd_nbricks)));
}

hipError_t launch_step(int store, bool odd, int bc, const StepArgs& a, hipStream_t s)
{
    if (!step_args_ok(store, a)) return hipErrorInvalidValue;
    switch (store) {
        case kStoreF64: return launch_step_store<StoreF64>(odd, bc, a, s);
        case kStoreF32: return launch_step_store<StoreF32>(odd, bc, a, s);
        case kStoreF16: return launch_step_store<StoreF16>(odd, bc, a, s);
        case kStoreBF16: return launch_step_store<StoreBF16>(odd, bc, a, s);
    }
    return hipErrorInvalidValue;
}

// Batched step: `host_table` (n entries, validated here) mirrors the device
// table; all instances share the store, block size and group width.
hipError_t launch_batch_step(int store, bool odd, const StepArgs* host_table, int n, const StepArgs* dev_table,
                             const int* dev_tile_inst, int ntiles, int xcd_remap, hipStream_t s)
{
    if (n < 1 || ntiles < 1) return hipErrorInvalidValue;
    int total = 0;
    for (int i = 0; i < n; ++i) {
        if (!step_args_ok(store, host_table[i]) || host_table[i].tile_begin != total) return hipErrorInvalidValue;
        if (host_table[i].tile_x != host_table[0].tile_x || host_table[i].vw != host_table[0].vw ||
            (host_table[i].nseg > 0) != (host_table[0].nseg > 0))
            return hipErrorInvalidValue;
        total += host_table[i].ntiles;
    }
    if (total != ntiles) return hipErrorInvalidValue;
    StepArgs a0 = host_table[0];
    a0.xcd_remap = xcd_remap;
    switch (store) {
        case kStoreF64: return launch_batch_store<StoreF64>(odd, a0, dev_table, dev_tile_inst, ntiles, s);
        case kStoreF32: return launch_batch_store<StoreF32>(odd, a0, dev_table, dev_tile_inst, ntiles, s);
        case kStoreF16: return launch_batch_store<StoreF16>(odd, a0, dev_table, dev_tile_inst, ntiles, s);
        case kStoreBF16: return launch_batch_store<StoreBF16>(odd, a0, dev_table, dev_tile_inst, ntiles, s);
    }
    return hipErrorInvalidValue;
}


// ------------------------------------------------------- statistics reduce

// Adds one sample of per-tile partial sums to the per-layer accumulator
// acc[y][8] (7 sums and the cell count), summing tiles in a fixed order.
__global__ __launch_bounds__(256) void k_stats_reduce(const double* __restrict__ part, int ntx, int ny, int nz, int nx,
                                                      double* __restrict__ acc)
{
    __shared__ double red[256][7];
    const int y = blockIdx.x;
    double s[7] = {0, 0, 0, 0, 0, 0, 0};
    const int per_layer = nz * ntx;
    for (int j = threadIdx.x; j < per_layer; j += blockDim.x) {
        const int z = j / ntx, xt = j - z * ntx;
        const long long t = (long long)xt + (long long)ntx * ((long long)y + (long long)ny * z);
#pragma unroll
        for (int k = 0; k < 7; ++k) s[k] += part[t * 7 + k];
    }
#pragma unroll
    for (int k = 0; k < 7; ++k) red[threadIdx.x][k] = s[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 7; ++k) red[threadIdx.x][k] += red[threadIdx.x + w][k];
        __syncthreads();
    }
    if (threadIdx.x < 7) acc[y * 8 + threadIdx.x] += red[0][threadIdx.x];
    if (threadIdx.x == 7) acc[y * 8 + 7] += (double)nx * (double)nz;
}

hipError_t launch_stats_reduce(const double* partials, int ntx, int ny, int nz, int nx, double* acc, hipStream_t s)
{
    hipLaunchKernelGGL(k_stats_reduce, dim3(ny), dim3(256), 0, s, partials, ntx, ny, nz, nx, acc);
    return hipGetLastError();
}

// ------------------------------------------------------------ initial state

// fpost(0) = f_eq(1, u0): u0 = profile(y) (1 + d0, d1, d2), d_i uniform in
// [-noise, noise) from splitmix64 counter 3 c + i; stored in layout P.
template <typename S>
__global__ __launch_bounds__(256) void k_init(void* hv, long long n, int nx, int ny, int nz, int brick,
                                              const double* __restrict__ prof, double noise, unsigned long long seed)
{
    using T = typename S::T;
    T* h = (T*)hv;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int x = (int)(c % nx);
    const int y = (int)((c / nx) % ny);
    const int z = (int)(c / ((long long)nx * ny));
    const long long m = cell_index(x, y, z, nx, ny, nz, brick);
    const double up = prof[y];
    double d[3];
    for (int i = 0; i < 3; ++i) d[i] = noise * (2.0 * uniform01(seed, 3ull * (unsigned long long)c + i) - 1.0);
    const double ux = up * (1.0 + d[0]), uy = up * d[1], uz = up * d[2];
    const double usq = 1.5 * (ux * ux + uy * uy + uz * uz);
    for_each_dir([&](auto A) {
        constexpr int a = decltype(A)::value;
        const double eu = kEx[a] * ux + kEy[a] * uy + kEz[a] * uz;
        const double heq = weight<double>(a) * (3.0 * eu + 4.5 * eu * eu - usq);
        h[(long long)opp(a) * n + m] = S::from_double(heq);
    });
}

// in[k][i], k = rho, u_x, u_y, u_z of cell c = first + i: the post-collision
// state f*(0) = f_eq(rho, u) of Eq. 1, stored as h = f - w in layout P.
template <typename S>
__global__ __launch_bounds__(256) void k_init_moments(void* hv, long long n, int nx, int ny, int nz, int brick,
                                                      long long first, long long count, const double* __restrict__ in)
{
    using T = typename S::T;
    T* h = (T*)hv;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const long long c = first + i;
    const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((long long)nx * ny));
    const long long m = cell_index(x, y, z, nx, ny, nz, brick);
    const double rho = in[i], ux = in[count + i], uy = in[2 * count + i], uz = in[3 * count + i];
    const double usq = 1.5 * (ux * ux + uy * uy + uz * uz);
    for_each_dir([&](auto A) {
        constexpr int a = decltype(A)::value;
        const double eu = kEx[a] * ux + kEy[a] * uy + kEz[a] * uz;
        const double heq = weight<double>(a) * ((rho - 1.0) + rho * (3.0 * eu + 4.5 * eu * eu - usq));
        h[(long long)opp(a) * n + m] = S::from_double(heq);
    });
}

// ------------------------------------------------- state in canonical form

// in[a][i]: h of the post-collision f*_a(c), c = first + i; written in layout P.
template <typename S>
__global__ __launch_bounds__(256) void k_set_state(void* hv, long long n, int nx, int ny, int nz, int brick,
                                                   long long first, long long count, const double* __restrict__ in)
{
    using T = typename S::T;
    T* h = (T*)hv;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const long long c = first + i;
    const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((long long)nx * ny));
    const long long m = cell_index(x, y, z, nx, ny, nz, brick);
    for (int a = 0; a < kQ; ++a) h[(long long)opp(a) * n + m] = S::from_double(in[(long long)a * count + i]);
}

struct Pos {
    int x, y, z;
};

__device__ __forceinline__ Pos cell_pos(long long c, int nx, int ny)
{
    Pos q;
    q.x = (int)(c % nx);
    const long long r = c / nx;
    q.y = (int)(r % ny);
    q.z = (int)(r / ny);
    return q;
}

// memory index of cell (x, y, z), x and z taken periodically
__device__ __forceinline__ long long cell_at(int x, int y, int z, int nx, int ny, int nz, int brick)
{
    x = (x % nx + nx) % nx;
    z = (z % nz + nz) % nz;
    return cell_index(x, y, z, nx, ny, nz, brick);
}

// out[a][i]: h of f*_a at cell i of the list (or first + i), from either layout.
template <typename S>
__global__ __launch_bounds__(256) void k_get_state(const void* hv, long long n, int nx, int ny, int nz, int brick,
                                                   int layout_s, int layout_spec, const long long* __restrict__ cells,
                                                   long long first, long long count, double* __restrict__ out,
                                                   const void* __restrict__ wn)
{
    using T = typename S::T;
    const T* h = (const T*)hv;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const long long c = cells ? cells[i] : first + i;
    const Pos q = cell_pos(c, nx, ny);
    const long long m = cell_index(q.x, q.y, q.z, nx, ny, nz, brick);
    for_each_dir([&](auto A) {
        constexpr int a = decltype(A)::value;
        if (wn) {
            // wall nodes: a first-layer population bound for the wall node at x + e_a waits
            // in the arrival ring of the latest step
            const int dy = q.y + kEy[a];
            if (dy < 0 || dy >= ny) {
                const bool tp = dy >= ny;
                const int k = tp ? in_index_b(mirror_y(opp(a))) : in_index_b(opp(a));
                const long long r = wn_index(layout_s, tp ? 1 : 0, k, (q.z + kEz[a] + nz) % nz, (q.x + kEx[a] + nx) % nx,
                                             nx, nz);
                out[(long long)a * count + i] = S::to_double(((const T*)wn)[r]);
                return;
            }
        }
        long long src;
        int slot;
        if (!layout_s) {
            slot = opp(a);
            src = m;
        } else {
            const int dy = q.y + kEy[a];
            if (dy >= 0 && dy < ny) {
                slot = a;
                src = cell_at(q.x + kEx[a], dy, q.z + kEz[a], nx, ny, nz, brick);
            } else if (!layout_spec || !is_tangential(a)) {
                slot = opp(a);
                src = m;
            } else {
                slot = mirror_y(a);
                src = cell_at(q.x + kEx[a], q.y, q.z + kEz[a], nx, ny, nz, brick);
            }
        }
        out[(long long)a * count + i] = S::to_double(h[(long long)slot * n + src]);
    });
}

// ---------------------------------------------------------------- observe

// Observables of the current state: the gather (and WFB) the next step would
// do, without any write.  mode 0: rho, u per cell.  mode 1: wall records per
// wall cell, i = w * nx * nz + z * nx + x (w = 0 bottom, 1 top).
template <typename S>
__global__ __launch_bounds__(256) void k_observe(ObsArgs p)
{
    using T = typename S::T;
    using R = typename S::R;
    const T* h = (const T*)p.h;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.count) return;
    long long c;
    int x, y, z;
    if (p.mode == 0) {
        const long long cc = p.cells ? p.cells[i] : p.first + i;
        const Pos q = cell_pos(cc, p.nx, p.ny);
        x = q.x; y = q.y; z = q.z;
    } else {
        const long long per = (long long)p.nx * p.nz;
        const int w = (int)(i / per);
        z = (int)((i % per) / p.nx);
        x = (int)(i % p.nx);
        y = w ? p.ny - 1 : 0;
    }
    c = cell_index(x, y, z, p.nx, p.ny, p.nz, p.brick);  // memory index
    const bool bot = (y == 0), top = (y == p.ny - 1);
    const long long n = p.n;
    R f[kQ];
    for_each_dir([&](auto A) {
        constexpr int a = decltype(A)::value;
        constexpr int ex = kEx[a], ey = kEy[a], ez = kEz[a];
        const int sy = y - ey;
        if (p.wall_nodes && (sy < 0 || sy >= p.ny)) {
            // what the wall node at x - e_a sends into the fluid next step
            const bool tp = sy >= p.ny;
            const int k = tp ? in_index_b(mirror_y(a)) : in_index_b(a);
            f[a] = S::load((const T*)p.wn + wn_index(2 + p.layout_s, tp ? 1 : 0, k, (z - ez + p.nz) % p.nz,
                                                     (x - ex + p.nx) % p.nx, p.nx, p.nz));
            return;
        }
        if (p.layout_s) {
            f[a] = S::load(h + (long long)a * n + c);
        } else {
            if (sy >= 0 && sy < p.ny) {
                f[a] = S::load(h + (long long)opp(a) * n + cell_at(x - ex, sy, z - ez, p.nx, p.ny, p.nz, p.brick));
            } else if (p.bc == kBB || !is_tangential(a)) {
                f[a] = S::load(h + (long long)a * n + c);
            } else {
                f[a] = S::load(h + (long long)opp(mirror_y(a)) * n + cell_at(x - ex, y, z - ez, p.nx, p.ny, p.nz, p.brick));
            }
        }
    });
    WallRecord rec{0.0, 0.0, 0.0, 0.0};
    int iters = 0;
    // Eq. B-1 per wall cell: the population sum after the wall correction minus
    // the sum before, both summed in direction order in the step's own precision
    // over the deviations h_a = f_a - w_a the step holds (the weights cancel)
    R sum0 = R(0);
    if (p.dmass) for_each_dir([&](auto A) { sum0 += f[decltype(A)::value]; });
    if (p.bc == kWFB && (bot || top) && !p.wall_nodes) {
        bool fail = false;
        rec = wfb_correct<R>(f, top, p.fx, p.y1, p.nu0, p.kappa, p.bconst, p.ekb, p.newton_tol, p.newton_maxit, iters,
                          fail);
        if (fail) iters = -iters;
    }
    if (p.dmass) {
        R sum1 = R(0);
        for_each_dir([&](auto A) { sum1 += f[decltype(A)::value]; });
        p.dmass[2 * i] = (double)(sum1 - sum0);
        p.dmass[2 * i + 1] = 1.0 + (double)sum0;
    }
    R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
    for_each_dir([&](auto A) {
        constexpr int a = decltype(A)::value;
        drho += f[a];
        if constexpr (kEx[a] != 0) jx += R(kEx[a]) * f[a];
        if constexpr (kEy[a] != 0) jy += R(kEy[a]) * f[a];
        if constexpr (kEz[a] != 0) jz += R(kEz[a]) * f[a];
    });
    const R rho = R(1) + drho;
    const R ux = (jx + R(0.5) * (R)p.fx) / rho, uy = jy / rho, uz = jz / rho;
    if (p.mode == 0) {
        if (p.out) {
            double* o = p.out + 4 * i;
            o[0] = (double)rho; o[1] = (double)ux; o[2] = (double)uy; o[3] = (double)uz;
        } else {
            if (p.soa[0]) p.soa[0][i] = (double)rho;
            if (p.soa[1]) p.soa[1][i] = (double)ux;
            if (p.soa[2]) p.soa[2][i] = (double)uy;
            if (p.soa[3]) p.soa[3][i] = (double)uz;
        }
        return;
    }
    if (p.wall_nodes) {
        // the stress the next wall-node collision applies (WFB, from the first
        // layer's record), the momentum exchange of the populations waiting to be
        // reversed there (bounce-back), nothing for free-slip
        const int wl = top ? 1 : 0;
        const double* r = p.wn_rec + (((long long)wl * p.nz + z) * p.nx + x) * 4;
        const double U = sqrt(r[1] * r[1] + r[2] * r[2]);
        rec = WallRecord{0.0, 0.0, 0.0, U};
        if (p.bc == kWFB) {
            rec = wall_record(r[0], r[1], r[2], U, r[3]);
        } else if (p.bc == kBB) {
            double tx = 0.0, tz = 0.0;
            for_each_dir([&](auto B) {
                constexpr int b = decltype(B)::value;
                if ((kEy[b] == -1 && !top) || (kEy[b] == 1 && top)) {
                    const int k = top ? in_index_b(mirror_y(opp(b))) : in_index_b(opp(b));
                    const double fb = S::to_double(((const T*)p.wn)[wn_index(p.layout_s, wl, k, z, x, p.nx, p.nz)]);
                    tx += -2.0 * kEx[b] * fb;
                    tz += -2.0 * kEz[b] * fb;
                }
            });
            rec.taux = tx;
            rec.tauz = tz;
            rec.utau = sqrt(sqrt(tx * tx + tz * tz) / r[0]);
        }
    } else if (p.bc == kBB) {
        // force on the fluid by momentum exchange: every population leaving through the
        // wall comes back reversed; f*_b sits in slot opp(b) of the cell in both layouts
        double tx = 0.0, tz = 0.0;
        for_each_dir([&](auto A) {
            constexpr int b = decltype(A)::value;
            const bool leaves = (kEy[b] == -1 && bot) || (kEy[b] == 1 && top);
            if (leaves) {
                const double fb = (double)S::load(h + (long long)opp(b) * n + c);
                tx += -2.0 * kEx[b] * fb;
                tz += -2.0 * kEz[b] * fb;
            }
        });
        rec.taux = tx;
        rec.tauz = tz;
        rec.utau = sqrt(sqrt(tx * tx + tz * tz) / (double)rho);
        rec.U = sqrt((double)ux * (double)ux + (double)uz * (double)uz);
    } else if (p.bc == kFreeSlip) {
        rec.U = sqrt((double)ux * (double)ux + (double)uz * (double)uz);
    }
    if (p.wall_nodes) iters = 0;
    if (p.out) {
        double* o = p.out + 4 * i;
        o[0] = rec.taux; o[1] = rec.tauz; o[2] = rec.utau; o[3] = rec.U;
    } else {
        if (p.soa[0]) p.soa[0][i] = rec.taux;
        if (p.soa[1]) p.soa[1][i] = rec.tauz;
        if (p.soa[2]) p.soa[2][i] = rec.utau;
        if (p.soa[3]) p.soa[3][i] = rec.U;
    }
    if (p.iters) p.iters[i] = iters;
}

// --------------------------------------------- re-reflection of a layout S

// When the boundary switches between bounce-back and mirror reflection after
// an odd number of steps, the wall-crossing populations already reflected by
// the old rule are moved to where the new rule puts them.  Pass 0 gathers the
// five outgoing populations of every wall cell into tmp, pass 1 scatters them.
template <typename S>
__global__ __launch_bounds__(256) void k_relayout(void* hv, long long n, int nx, int ny, int nz, int brick,
                                                  int from_spec, int to_spec, double* __restrict__ tmp, int pass)
{
    using T = typename S::T;
    T* h = (T*)hv;
    const long long per = (long long)nx * nz;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * per) return;
    const int w = (int)(i / per);
    const int z = (int)((i % per) / nx), x = (int)(i % nx);
    const int y = w ? ny - 1 : 0;
    const long long c = cell_index(x, y, z, nx, ny, nz, brick);
    const int spec = pass == 0 ? from_spec : to_spec;
    int k = 0;
    for_each_dir([&](auto A) {
        constexpr int b = decltype(A)::value;
        if ((w == 0 && kEy[b] == -1) || (w == 1 && kEy[b] == 1)) {
            long long slot;
            if (!spec || !is_tangential(b))
                slot = (long long)opp(b) * n + c;
            else
                slot = (long long)mirror_y(b) * n + cell_at(x + kEx[b], y, z + kEz[b], nx, ny, nz, brick);
            if (pass == 0)
                tmp[i * 5 + k] = S::to_double(h[slot]);
            else
                h[slot] = S::from_double(tmp[i * 5 + k]);
            ++k;
        }
    });
}

// ----------------------------------------------------------- misc kernels

// The bandwidth reference: a streaming copy, 16 bytes per lane per access,
// non-temporal both ways.  Each block copies one contiguous 16 KB chunk (four
// accesses per lane, all loads before the stores); the blocks go to the XCDs
// in chunks of consecutive tiles, as the step kernels' do (measured on
// MI355X: 6.0-6.3 TB/s against 5.3 for chunks striding over the buffer and
// 5.9 for the plain block order).  dst may equal src: the in-place pass is the
// AA step's own access form.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy(const u32x4* src, u32x4* dst, long long n)
{
    const long long base = (long long)tile_of_block((int)blockIdx.x, (int)gridDim.x, kXcdChunkLog2 + 1) * 1024;
    const long long i = base + threadIdx.x;
    u32x4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const long long j = i + k * 256;
        if (j < n) v[k] = __builtin_nontemporal_load(src + j);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const long long j = i + k * 256;
        if (j < n) __builtin_nontemporal_store(v[k], dst + j);
    }
}

__global__ __launch_bounds__(256) void k_wall_utau(const double* __restrict__ U, int n, double y1, double nu,
                                                   double kappa, double bconst, double ekb, double tol, int maxit,
                                                   double* __restrict__ ut, int* __restrict__ iters)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int it = 0;
    bool fail = false;
    double r = 0.0;
    if (U[i] > 0.0) r = wall_utau(U[i], y1, nu, kappa, bconst, ekb, tol, maxit, it, fail);
    ut[i] = fail ? -1.0 : r;
    iters[i] = it;
}

// Store-format round trip through the same group codec the step kernels use:
// out[i] = decode(encode(in[i])), groups of the widest width for the format.
template <typename S>
__global__ __launch_bounds__(256) void k_codec(const float* __restrict__ in, float* __restrict__ out, long long n)
{
    constexpr int V = 8 / (int)sizeof(typename S::T);
    using Ln = Lane<S, V>;
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g * V >= n) return;
    u32x2 w{0u, 0u};
#pragma unroll
    for (int k = 0; k < V; ++k)
        if (g * V + k < n) Ln::set(w, k, (typename S::R)in[g * V + k]);
#pragma unroll
    for (int k = 0; k < V; ++k)
        if (g * V + k < n) out[g * V + k] = (float)Ln::get(w, k);
}

// ------------------------------------------------------------- wall nodes

// Wall nodes of a state set from outside (layout P), one thread per wall
// node (x, z) of wall w = i / (nx nz): the record of the first-layer cell
// below (above) it, from the plain moments of its post-collision populations
// (rho = sum f, u = sum e f / rho) and Spalding's law; the populations its
// in-plane neighbours x - e_b send towards it (arrival ring 0); and one
// wall-node collision of them (output ring 2), as if the state had also been
// the previous step's.
template <typename S>
__global__ __launch_bounds__(256) void k_node_start(StepArgs p)
{
    using T = typename S::T;
    const T* h = (const T*)p.h;
    T* wn = (T*)p.wn;
    const long long per = (long long)p.nx * p.nz;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * per) return;
    const int wl = (int)(i / per);
    const int z = (int)((i % per) / p.nx), x = (int)(i % p.nx);
    const int y = wl ? p.ny - 1 : 0;
    const long long n = p.n;
    const long long c = cell_index(x, y, z, p.nx, p.ny, p.nz, p.brick);
    double drho = 0.0, jx = 0.0, jz = 0.0;
    for_each_dir([&](auto A) {
        constexpr int a = decltype(A)::value;
        const double v = S::to_double(h[(long long)opp(a) * n + c]);
        drho += v;
        if constexpr (kEx[a] != 0) jx += kEx[a] * v;
        if constexpr (kEz[a] != 0) jz += kEz[a] * v;
    });
    const double rho = 1.0 + drho, ux = jx / rho, uz = jz / rho;
    const double U[1] = {sqrt(ux * ux + uz * uz)};
    double ut[1];
    int it = 0;
    bool fail = false;
    wall_utau_n<1>(U, p.y1, p.nu0, p.kappa, p.bconst, p.ekb, p.newton_tol, p.newton_maxit, ut, it, fail);
    if (fail) {
        atomicOr(&p.flags->status, 2);
        atomicMin(&p.flags->first_bad, 0ull);
    }
    double* r = p.wn_rec + (((long long)wl * p.nz + z) * p.nx + x) * 4;
    r[0] = rho; r[1] = ux; r[2] = uz; r[3] = ut[0];
    double arr[5];
    for_each_dir([&](auto B) {
        constexpr int b = decltype(B)::value;
        if ((kEy[b] == -1 && wl == 0) || (kEy[b] == 1 && wl == 1)) {
            const int k = wl ? in_index_b(mirror_y(opp(b))) : in_index_b(opp(b));
            const long long src = cell_index((x - kEx[b] + p.nx) % p.nx, y, (z - kEz[b] + p.nz) % p.nz, p.nx, p.ny,
                                             p.nz, p.brick);
            const T v = h[(long long)opp(b) * n + src];
            wn[wn_index(0, wl, k, z, x, p.nx, p.nz)] = v;
            arr[k] = S::to_double(v);
        }
    });
    const WallRecord rec = wall_record(rho, ux, uz, U[0], ut[0]);
    const bool wfb = (p.bc == kWFB), bb = (p.bc == kBB);
    for (int k = 0; k < 5; ++k) {
        double v = arr[bb ? k : node_spec(k)];
        if (wfb) {
            if (k == 1) v += 0.5 * rec.taux;
            else if (k == 3) v -= 0.5 * rec.taux;
            else if (k == 2) v += 0.5 * rec.tauz;
            else if (k == 4) v -= 0.5 * rec.tauz;
        }
        wn[wn_index(2, wl, k, z, x, p.nx, p.nz)] = S::from_double(v);
    }
}

// out[w][k][z][x] = output ring 2 + slot as doubles
template <typename S>
__global__ __launch_bounds__(256) void k_node_get(const void* wn, int slot, int nx, int nz, double* __restrict__ out)
{
    using T = typename S::T;
    const long long m = 10ll * nx * nz;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    out[i] = S::to_double(((const T*)wn)[wn_index(2 + slot, 0, 0, 0, 0, nx, nz) + i]);
}

// ---------------------------------------------------------------- launchers

template <template <typename> class K, typename... Args>
static hipError_t dispatch_store(int store, dim3 g, dim3 b, hipStream_t s, Args... args)
{
    switch (store) {
        case kStoreF64: hipLaunchKernelGGL(K<StoreF64>::fn, g, b, 0, s, args...); break;
        case kStoreF32: hipLaunchKernelGGL(K<StoreF32>::fn, g, b, 0, s, args...); break;
        case kStoreF16: hipLaunchKernelGGL(K<StoreF16>::fn, g, b, 0, s, args...); break;
        case kStoreBF16: hipLaunchKernelGGL(K<StoreBF16>::fn, g, b, 0, s, args...); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename S> struct InitK { static constexpr auto fn = k_init<S>; };
template <typename S> struct SetK { static constexpr auto fn = k_set_state<S>; };
template <typename S> struct InitMK { static constexpr auto fn = k_init_moments<S>; };
template <typename S> struct GetK { static constexpr auto fn = k_get_state<S>; };
template <typename S> struct ObsK { static constexpr auto fn = k_observe<S>; };
template <typename S> struct RelK { static constexpr auto fn = k_relayout<S>; };
template <typename S> struct CodecK { static constexpr auto fn = k_codec<S>; };
template <typename S> struct NodeStartK { static constexpr auto fn = k_node_start<S>; };
template <typename S> struct NodeGetK { static constexpr auto fn = k_node_get<S>; };

static dim3 blocks_for(long long n, int bs) { return dim3((unsigned)((n + bs - 1) / bs)); }

hipError_t launch_init_spalding(int store, void* h, long long n, int nx, int ny, int nz, int brick,
                                const double* profile, double noise, unsigned long long seed, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    return dispatch_store<InitK>(store, blocks_for(n, 256), dim3(256), s, h, n, nx, ny, nz, brick, profile, noise,
                                 seed);
}

hipError_t launch_set_state(int store, void* h, long long n, int nx, int ny, int nz, int brick, long long first,
                            long long count, const double* in, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    return dispatch_store<SetK>(store, blocks_for(count, 256), dim3(256), s, h, n, nx, ny, nz, brick, first, count,
                                in);
}

hipError_t launch_init_moments(int store, void* h, long long n, int nx, int ny, int nz, int brick, long long first,
                               long long count, const double* in, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    return dispatch_store<InitMK>(store, blocks_for(count, 256), dim3(256), s, h, n, nx, ny, nz, brick, first, count,
                                  in);
}

hipError_t launch_get_state(int store, const void* h, long long n, int nx, int ny, int nz, int brick, int layout_s,
                            int layout_spec, const long long* cells, long long first, long long count, double* out,
                            const void* wn, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    return dispatch_store<GetK>(store, blocks_for(count, 256), dim3(256), s, h, n, nx, ny, nz, brick, layout_s,
                                layout_spec, cells, first, count, out, wn);
}

hipError_t launch_node_start(int store, const StepArgs& a, hipStream_t s)
{
    if (!a.wall_nodes || !a.wn || !a.wn_rec) return hipErrorInvalidValue;
    const long long m = 2ll * a.nx * a.nz;
    return dispatch_store<NodeStartK>(store, blocks_for(m, 256), dim3(256), s, a);
}

hipError_t launch_node_get(int store, const void* wn, int slot, int nx, int nz, double* out, hipStream_t s)
{
    if (!wn || slot < 0 || slot > 1) return hipErrorInvalidValue;
    return dispatch_store<NodeGetK>(store, blocks_for(10ll * nx * nz, 256), dim3(256), s, wn, slot, nx, nz, out);
}

hipError_t launch_observe(int store, const ObsArgs& a, hipStream_t s)
{
    if (a.count <= 0) return hipSuccess;
    return dispatch_store<ObsK>(store, blocks_for(a.count, 256), dim3(256), s, a);
}

hipError_t launch_relayout(int store, void* h, long long n, int nx, int ny, int nz, int brick, int from_spec,
                           int to_spec, double* tmp, hipStream_t s)
{
    const long long m = 2ll * nx * nz;
    hipError_t e = dispatch_store<RelK>(store, blocks_for(m, 256), dim3(256), s, h, n, nx, ny, nz, brick, from_spec,
                                        to_spec, tmp, 0);
    if (e != hipSuccess) return e;
    return dispatch_store<RelK>(store, blocks_for(m, 256), dim3(256), s, h, n, nx, ny, nz, brick, from_spec, to_spec,
                                tmp, 1);
}

hipError_t launch_codec(int store, const float* in, float* out, long long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    // one thread per group; n threads cover the narrowest (one-element) groups
    return dispatch_store<CodecK>(store, blocks_for(n, 256), dim3(256), s, in, out, n);
}

// First-layer y+ of the wall records (Fig. 7): y+ = y1 u_tau / nu0 per wall
// cell, from the friction velocities ut[m].  k_yplus_moments: one block clears
// the nbins + 2 counters, then forms the mean and the mean square deviation
// in FP64 in a fixed order (thread t takes cells t, t + 256, ...; then a tree
// over the threads) and writes the mean and the population standard
// deviation.  k_yplus_hist counts z = (y+ - mean) / std into nbins bins of
// width (hi - lo) / nbins from lo, with an underflow bin first and an overflow
// bin last.
__global__ __launch_bounds__(256) void k_yplus_moments(const double* __restrict__ ut, long long m, double y1,
                                                       double nu0, double* __restrict__ ms, int nbins,
                                                       unsigned long long* __restrict__ counts)
{
    __shared__ double sh[256];
    const int t = (int)threadIdx.x;
    for (int b = t; b < nbins + 2; b += 256) counts[b] = 0ull;
    // two passes: the mean, then the mean square deviation from it
    double mean = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        double a = 0.0;
        for (long long i = t; i < m; i += 256) {
            const double yp = (y1 * ut[i]) / nu0;
            a += pass == 0 ? yp : (yp - mean) * (yp - mean);
        }
        sh[t] = a;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o) sh[t] += sh[t + o];
            __syncthreads();
        }
        const double v = sh[0] / (double)m;
        __syncthreads();
        if (pass == 0) {
            mean = v;
        } else if (t == 0) {
            ms[0] = mean;
            ms[1] = sqrt(v);
        }
    }
}

__global__ __launch_bounds__(256) void k_yplus_hist(const double* __restrict__ ut, long long m, double y1, double nu0,
                                                    const double* __restrict__ ms, double lo, double scale, int nbins,
                                                    unsigned long long* __restrict__ counts)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const double yp = (y1 * ut[i]) / nu0;
    const double z = (yp - ms[0]) / ms[1];
    const double u = (z - lo) * scale;
    int bin;
    if (!(u >= 0.0)) bin = 0;                 // below lo (and NaN)
    else if (u >= (double)nbins) bin = nbins + 1;
    else bin = 1 + (int)floor(u);
    atomicAdd(&counts[bin], 1ull);
}

hipError_t launch_yplus_pdf(const double* ut, long long m, double y1, double nu0, double* ms, double lo, double scale,
                            int nbins, unsigned long long* counts, hipStream_t s)
{
    if (m <= 0 || nbins < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_yplus_moments, dim3(1), dim3(256), 0, s, ut, m, y1, nu0, ms, nbins, counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_yplus_hist, blocks_for(m, 256), dim3(256), 0, s, ut, m, y1, nu0, ms, lo, scale, nbins,
                       counts);
    return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s)
{
    if (bytes % 16 != 0) return hipErrorInvalidValue;
    const long long n = (long long)(bytes / 16);
    if (n == 0) return hipSuccess;
    // one 16 KB chunk per block
    const long long blocks = (n + 1023) / 1024;
    if (blocks >= (1ll << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, (const u32x4*)src, (u32x4*)dst, n);
    return hipGetLastError();
}

hipError_t launch_wall_utau(const double* U, int n, double y1, double nu, double kappa, double bconst, double tol,
                            int maxit, double* utau, int* iters, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_wall_utau, blocks_for(n, 256), dim3(256), 0, s, U, n, y1, nu, kappa, bconst,
                       exp(-kappa * bconst), tol, maxit, utau, iters);
    return hipGetLastError();
}


}  // namespace lbmwf
