// Internal interface between the C-ABI (lbm_capi.hip) and the device kernels
// (lbm_kernels.hip; the step kernels in lbm_step.h, instantiated per store in
// step_*.hip).  Not installed; the public interface is include/lbmwf.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmwf {

// Device-side status, one per context (or batch).
struct DevFlags {
    int status;                    // bit 0: non-finite or non-positive density; bit 1: Newton cap
    int max_newton_iters;          // largest Newton iteration count seen at a wall cell
    unsigned long long first_bad;  // smallest step index that raised a status bit
    long long cnt[2];              // step index of the next odd-kernel [1] / even-kernel [0] launch
};

enum Boundary { kBB = 0, kWFB = 1, kFreeSlip = 2 };

// Population layout on the device: slot a holds N = nx ny nz values; within
// a slot, x-rows are grouped in bricks of `brick` consecutive y (the last
// brick may be shorter), ordered [y / brick][z][y % brick][x].  brick = ny is
// the plain [z][y][x] order.  Neighbouring z-planes of a brick lie brick rows
// apart instead of a whole plane, which keeps the shifted accesses of a step
// close to each other in memory.
__host__ __device__ inline long long row_index(int y, int z, int ny, int nz, int brick)
{
    const int yb = y / brick, yi = y - yb * brick;
    const int bk = (ny - yb * brick) < brick ? (ny - yb * brick) : brick;
    return (long long)yb * brick * nz + (long long)z * bk + yi;
}

__host__ __device__ inline long long cell_index(int x, int y, int z, int nx, int ny, int nz, int brick)
{
    return row_index(y, z, ny, nz, brick) * nx + x;
}

// Division by a launch constant d as a multiply and a shift: for 0 <= n < 2^31,
// n / d == (n m) >> s with s = 31 + ceil(log2 d), m = floor(2^s / d) + 1
// (Granlund & Montgomery 1994, Thm. 4.2: 2^s < m d <= 2^s + 2^(s-31)).
struct FastDiv {
    unsigned long long m;
    int s;
};

inline FastDiv make_fastdiv(int d)
{
    int l = 0;
    while ((1ll << l) < d) ++l;
    FastDiv f;
    f.s = 31 + l;
    f.m = ((1ull << f.s) / (unsigned long long)d) + 1;
    return f;
}

__host__ __device__ inline int fdiv(int n, FastDiv f) { return (int)(((unsigned long long)n * f.m) >> f.s); }

// Parameters of one fused step launch (or of one instance of a batched
// launch).  A block processes one tile: rpb whole x-rows of one z-plane, or
// one segment of tile_x * vw cells of a single x-row.  Tiles are numbered in
// memory order: x segment, row group within a brick, z, brick.
enum { kBGK = 0, kMRT = 1 };

// Blocks go round-robin to the 8 XCDs; with the XCD remap each XCD takes
// chunks of 2^kXcdChunkLog2 consecutive tiles in turn.
constexpr int kXcdChunkLog2 = 5;

struct StepArgs {
    void* h;              // populations h_a = f_a - w_a, bricked layout (row_index)
    long long n;          // cells
    int nx, ny, nz;
    int brick;            // rows per brick (1 <= brick <= ny; rpb > 1 needs brick == ny)
    int bgroups;          // row groups per brick (brick / rpb, or nyt for a single brick)
    int nbricks;          // bricks (the last one may hold fewer groups)
    int bg_last;          // row groups of the last brick
    FastDiv fd_ntx, fd_brick_tiles, fd_bgroups, fd_bg_last, fd_tpr;  // tile and thread decomposition
    int spread;           // launch order: log2 of the tile chunks that cycle over the bricks (-1: memory order)
    int spread_rot;       // rotate the brick of each round of chunks by the round (brick count shares a factor with 8)
    int tiles_per_brick;  // tiles of one brick (every brick whole when spread >= 0)
    FastDiv fd_nbricks;
    int nseg;             // odd step by rows: each wavefront walks one row in nseg segments of 64 vw
                          // cells (tile_x / 64 rows per block); 0: the tile kernel
    int tile_x;           // threads per block
    int vw;               // cells per thread (1, 2 or 4): a group of vw * sizeof(store) <= 8 bytes
    int ntx;              // x segments per row (1: a block holds whole rows)
    int rpb;              // whole rows per block (1 when rows are split into segments)
    int nyt;              // row groups along y per z-plane
    int ntiles;           // tiles (= blocks) of this instance
    int tile_begin;       // first tile of this instance in a batched launch
    int bc;               // boundary (read by batched launches)
    int xcd_remap;        // 0: tile = block; c + 1: XCDs take chunks of 2^c tiles in turn
    int newton_maxit;
    double tau0;          // molecular relaxation time
    double cs2_18;        // 18 Cs^2 (Smagorinsky closure)
    const double* cs2_row;// 18 Cs^2 per row y with the van Driest damping; nullptr: cs2_18 in every row
    int coll;             // collision: kBGK or kMRT
    double mrt_s[5];      // MRT rates: energy, energy square, heat flux, fourth-order normal stress, third order
    double fx;            // body force density along x
    double y1;            // wall distance of the first layer used in y+
    double nu0;           // molecular viscosity (tau0 - 1/2) / 3
    double kappa, bconst; // Spalding's law constants
    double ekb;           // exp(-kappa B)
    double newton_tol;
    DevFlags* flags;
    double* partials;     // [nz][ny][ntx][7] statistics partial sums; nullptr on steps not sampled
    // wall nodes (wall_nodes = 1): the wall grid as a lattice node one spacing
    // outside the first fluid layer (see wn_index); bc is then the reflection
    // made at the wall nodes
    int wall_nodes;
    void* wn;             // four rings of the store type, wn_index
    double* wn_rec;       // [2 walls][nz][nx][4]: first layer's rho, u_x, u_z and u_tau of the latest step
};

// Wall-node rings, each [2 walls][5][nz][nx] elements of the store type:
//   ring s (s = 0, 1): the populations the first layer sent towards the wall
//     nodes, written by the step kernel of parity s (odd kernel: 1, even: 0;
//     initialisation: 0), element k of wall node (x, z) holding the
//     population arriving from direction opp(IN_k) (its reversal is IN_k);
//   ring 2 + s: what the wall nodes send into the fluid, written by the
//     kernel of parity s, element k being direction IN_k.
// IN_k = 3, 7, 11, 14, 17 at the bottom wall (e_y = +1), their mirror images
// 4, 13, 18, 8, 12 at the top.
__host__ __device__ inline long long wn_index(int ring, int w, int k, int z, int x, int nx, int nz)
{
    return ((((long long)ring * 2 + w) * 5 + k) * nz + z) * (long long)nx + x;
}

struct ObsArgs {
    const void* h;
    long long n;
    int nx, ny, nz;
    int brick;            // rows per brick of the population layout
    int layout_s;         // 0: post-collision layout (after an even number of steps), 1: streamed
    int bc;               // boundary used for the reflections still to be made
    int layout_spec;      // reflections already made (streamed layout) were mirror images
    int newton_maxit;
    double fx, y1, nu0, kappa, bconst, ekb, newton_tol;
    const long long* cells;  // optional cell list (nullptr: cells first .. first + count)
    long long first, count;
    double* out;          // [count][4]: rho, ux, uy, uz (mode 0); tau_x, tau_z, u_tau, U (mode 1, wall cells)
    double* soa[4];       // without out: the same four values of item i at index i of each non-null
                          // array (device memory)
    int* iters;           // optional, mode 1: Newton iterations per wall cell
    double* dmass;        // optional, mode 1: [count][2] = change of the population sum made
                          // by the wall correction, rho before it (Eq. B-1)
    int mode;
    int wall_nodes;       // the state has wall nodes (StepArgs::wall_nodes)
    const void* wn;       // their rings (wn_index) and records
    const double* wn_rec;
};

// launchers (lbm_kernels.hip); each returns the launch status
int step_vector_width(int store, int nx);
void step_geometry(int nx, int ny, int nz, int tile_x, int vw, int brick, StepArgs& a);
bool rows_ok(int nx, int vw);
void step_geometry_rows(int nx, int ny, int nz, int tile_x, int vw, int brick, StepArgs& a);
void set_spread(StepArgs& a, int log2);
bool brick_ok(int ny, int brick, int rpb);
hipError_t launch_batch_step(int store, bool odd, const StepArgs* host_table, int n, const StepArgs* dev_table,
                             const int* dev_tile_inst, int ntiles, int xcd_remap, hipStream_t s);
bool step_vector_width_ok(int store, int nx, int vw);
hipError_t launch_step(int store, bool odd, int bc, const StepArgs& a, hipStream_t s);
hipError_t launch_stats_reduce(const double* partials, int ntx, int ny, int nz, int nx, double* acc, hipStream_t s);
hipError_t launch_init_spalding(int store, void* h, long long n, int nx, int ny, int nz, int brick,
                                const double* profile, double noise, unsigned long long seed, hipStream_t s);
hipError_t launch_set_state(int store, void* h, long long n, int nx, int ny, int nz, int brick, long long first,
                            long long count, const double* in, hipStream_t s);
hipError_t launch_init_moments(int store, void* h, long long n, int nx, int ny, int nz, int brick, long long first,
                               long long count, const double* in, hipStream_t s);
hipError_t launch_get_state(int store, const void* h, long long n, int nx, int ny, int nz, int brick, int layout_s,
                            int layout_spec, const long long* cells, long long first, long long count, double* out,
                            const void* wn, hipStream_t s);
hipError_t launch_observe(int store, const ObsArgs& a, hipStream_t s);
// y+ distribution of m >= 1 wall cells from their friction velocities ut[m];
// clears counts[nbins + 2] itself, writes ms[2] = mean, standard deviation
hipError_t launch_yplus_pdf(const double* ut, long long m, double y1, double nu0, double* ms, double lo, double scale,
                            int nbins, unsigned long long* counts, hipStream_t s);
hipError_t launch_relayout(int store, void* h, long long n, int nx, int ny, int nz, int brick, int from_spec,
                           int to_spec, double* tmp, hipStream_t s);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
// wall nodes of a state set from outside (layout P): the first layer's plain
// moments and friction velocity, its wall-bound populations in arrival ring 0
// and one wall-node collision of them in output ring 2 (bc: the reflection)
hipError_t launch_node_start(int store, const StepArgs& a, hipStream_t s);
// the wall-node state for observation: outputs of ring 2 + slot as h = f - w,
// [2][5][nz][nx] doubles
hipError_t launch_node_get(int store, const void* wn, int slot, int nx, int nz, double* out, hipStream_t s);
hipError_t launch_codec(int store, const float* in, float* out, long long n, hipStream_t s);
// per-store step launchers (lbm_step.h), dispatched by launch_step / launch_batch_step
template <typename S>
hipError_t launch_step_store(bool odd, int bc, const StepArgs& a, hipStream_t s);
template <typename S>
hipError_t launch_batch_store(bool odd, const StepArgs& a0, const StepArgs* table, const int* tile_inst, int ntiles,
                              hipStream_t s);

hipError_t launch_wall_utau(const double* U, int n, double y1, double nu, double kappa, double bconst, double tol,
                            int maxit, double* utau, int* iters, hipStream_t s);

}  // namespace lbmwf
