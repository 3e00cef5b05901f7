// Internal interface between the C-ABI (lbm_capi.hip) and the device kernels
// (lbm_kernels.hip).  Not installed; the public interface is include/lbmwf.h.
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

// Parameters of one fused step launch (or of one instance of a batched
// launch).  A block processes one tile: rpb whole x-rows of one z-plane, or
// one segment of tile_x * vw cells of a single x-row.
struct StepArgs {
    void* h;              // populations h_a = f_a - w_a, [a][z][y][x]
    long long n;          // cells
    int nx, ny, nz;
    int tile_x;           // threads per block
    int vw;               // cells per thread (1, 2 or 4): a group of vw * sizeof(store) <= 8 bytes
    int ntx;              // x segments per row (1: a block holds whole rows)
    int rpb;              // whole rows per block (1 when rows are split into segments)
    int nyt;              // row groups along y per z-plane
    int ntiles;           // tiles (= blocks) of this instance
    int tile_begin;       // first tile of this instance in a batched launch
    int bc;               // boundary (read by batched launches)
    int xcd_remap;        // 1: give each XCD a contiguous range of tiles
    int newton_maxit;
    double tau0;          // molecular relaxation time
    double cs2_18;        // 18 Cs^2 (Smagorinsky closure)
    double fx;            // body force density along x
    double y1;            // wall distance of the first layer used in y+
    double nu0;           // molecular viscosity (tau0 - 1/2) / 3
    double kappa, bconst; // Spalding's law constants
    double ekb;           // exp(-kappa B)
    double newton_tol;
    DevFlags* flags;
    double* partials;     // [nz][ny][ntx][7] statistics partial sums; nullptr on steps not sampled
};

struct ObsArgs {
    const void* h;
    long long n;
    int nx, ny, nz;
    int layout_s;         // 0: post-collision layout (after an even number of steps), 1: streamed
    int bc;               // boundary used for the reflections still to be made
    int layout_spec;      // reflections already made (streamed layout) were mirror images
    int newton_maxit;
    double fx, y1, nu0, kappa, bconst, ekb, newton_tol;
    const long long* cells;  // optional cell list (nullptr: cells first .. first + count)
    long long first, count;
    double* out;          // [count][4]: rho, ux, uy, uz      (mode 0)
                          // [count][4]: tau_x, tau_z, u_tau, U (mode 1, wall cells)
    int* iters;           // optional, mode 1: Newton iterations per wall cell
    int mode;
};

// launchers (lbm_kernels.hip); each returns the launch status
int step_vector_width(int store, int nx);
void step_geometry(int nx, int ny, int nz, int tile_x, int vw, StepArgs& a);
hipError_t launch_batch_step(int store, bool odd, const StepArgs* host_table, int n, const StepArgs* dev_table,
                             const int* dev_tile_inst, int ntiles, int xcd_remap, hipStream_t s);
bool step_vector_width_ok(int store, int nx, int vw);
hipError_t launch_step(int store, bool odd, int bc, const StepArgs& a, hipStream_t s);
hipError_t launch_stats_reduce(const double* partials, int ntx, int ny, int nz, int nx, double* acc, hipStream_t s);
hipError_t launch_init_spalding(int store, void* h, long long n, int nx, int ny, int nz, const double* profile,
                                double noise, unsigned long long seed, hipStream_t s);
hipError_t launch_set_state(int store, void* h, long long n, long long first, long long count, const double* in,
                            hipStream_t s);
hipError_t launch_get_state(int store, const void* h, long long n, int nx, int ny, int nz, int layout_s,
                            int layout_spec, const long long* cells, long long first, long long count, double* out,
                            hipStream_t s);
hipError_t launch_observe(int store, const ObsArgs& a, hipStream_t s);
hipError_t launch_relayout(int store, void* h, long long n, int nx, int ny, int nz, int from_spec, int to_spec,
                           double* tmp, hipStream_t s);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
hipError_t launch_codec(int store, const float* in, float* out, long long n, hipStream_t s);
hipError_t launch_wall_utau(const double* U, int n, double y1, double nu, double kappa, double bconst, double tol,
                            int maxit, double* utau, int* iters, hipStream_t s);

}  // namespace lbmwf
