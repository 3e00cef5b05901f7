/*
 * lbmwf.h -- C ABI of the wall-function-bounce LBM-LES channel library.
 *
 * Method: Han, Ooka & Kikumoto, "A wall function approach in lattice
 * Boltzmann method: algorithm and validation using turbulent channel flow"
 * (arXiv 2009.04352).  One time step of a D3Q19 channel (x streamwise and
 * periodic, y wall-normal with a wall below the first and above the last
 * layer, z spanwise and periodic) is one fused GPU update:
 *   streaming of Eq. 1 with wall reflections (bounce-back, Eq. 3 in 3-D form;
 *   mirror reflection, Eq. 4 in 3-D form), the wall-function bounce (WFB)
 *   correction of Eq. 13-15 with tau_w from Spalding's law (Eq. 16-17) solved
 *   by Newton's method (Sec. 2.3), the moments of Eq. 2, a Smagorinsky eddy
 *   viscosity (Sec. 3.1) and BGK relaxation with the body force term F_a of
 *   Eq. 1.
 *
 * Units are lattice units: dx = dt = 1, reference density 1.  Host arrays of
 * populations are [a][z][y][x] with x fastest; cell index c = x + nx (y + ny z).
 * Directions a = 0..18 follow Table A-1.  The device array bound with
 * lbm_bind_storage is internal: 19 slots of nx ny nz values whose rows are
 * grouped in bricks of LBM_P_BRICK consecutive y, ordered
 * [y / brick][z][y % brick][x] (brick = ny: the plain [z][y][x] order);
 * lbm_get_state / lbm_set_state convert.
 *
 * Conventions for every function returning int:
 *   - LBM_OK (0) on success, a negative LBM_E_* code otherwise;
 *   - no exception, abort or exit ever crosses this boundary;
 *   - output arrays are written only on success;
 *   - a context is not thread-safe; distinct contexts are independent;
 *   - device work is enqueued on the context's stream (lbm_set_stream) and is
 *     asynchronous unless the function says it synchronises.
 */
#ifndef LBMWF_H
#define LBMWF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LBM_OK 0
#define LBM_E_ARG (-1)        /* an argument is out of range or a pointer is NULL */
#define LBM_E_STATE (-2)      /* call not valid in the context's state (e.g. no storage bound) */
#define LBM_E_OOM (-3)        /* a library-side allocation failed */
#define LBM_E_DEVICE (-4)     /* a HIP runtime call failed; lbm_last_error() has its text */
#define LBM_E_NONFINITE (-5)  /* a cell's density became non-finite or non-positive */
#define LBM_E_NEWTON (-6)     /* the wall-function Newton solve hit its iteration cap */

/* wall boundaries (Sec. 2.1-2.2) */
#define LBM_BB 0        /* bounce-back, the no-slip comparison path (Eq. 3, 3-D form) */
#define LBM_WFB 1       /* wall-function bounce (Eq. 14 with tau_w from Eq. 15-17) */
#define LBM_FREESLIP 2  /* mirror reflection (Eq. 4, 3-D form): WFB with tau_w = 0 */

/* storage formats of h_a = f_a - w_a */
#define LBM_STORE_F64 0   /* FP64 storage, FP64 arithmetic */
#define LBM_STORE_F32 1   /* FP32 storage, FP32 arithmetic (Newton in FP64) */
#define LBM_STORE_F16 2   /* IEEE binary16 storage, FP32 arithmetic */
#define LBM_STORE_BF16 3  /* bfloat16 storage, FP32 arithmetic */

/* parameter keys for lbm_set_param / lbm_get_param */
#define LBM_P_Y1 0            /* wall distance of the first layer in y+ = y1 u_tau / nu (default 1) */
#define LBM_P_NEWTON_TOL 1    /* Newton stops when |p_{k+1} - p_k| <= tol p_{k+1} (default 1e-14) */
#define LBM_P_NEWTON_MAXIT 2  /* Newton iteration cap (default 100) */
#define LBM_P_STATS_EVERY 3   /* sample plane statistics on steps t with t % k == 0; 0 = off (default) */
#define LBM_P_STORE 4         /* LBM_STORE_*; settable only before lbm_bind_storage (default F64) */
#define LBM_P_TILE_ODD 5      /* threads per block of the odd-step kernel: 64, 128, 256 or 512 */
#define LBM_P_TILE_EVEN 6     /* threads per block of the even-step kernel */
#define LBM_P_XCD_REMAP 7     /* 1: the 8 XCDs take chunks of consecutive tiles in turn (default; the chunk is
                               * LBM_P_XCD_CHUNK, 32 tiles by default), 0: identity */
#define LBM_P_GRAPH_STEPS 8   /* steps per captured HIP graph chunk; 0 = launch eagerly (default 32) */
#define LBM_P_BC 9            /* read-only here: the current boundary */
#define LBM_P_TAU0 10         /* read-only: molecular relaxation time */
#define LBM_P_FX 11           /* body force density along x; settable at any time */
#define LBM_P_CS 12           /* Smagorinsky constant; settable at any time */
#define LBM_P_VECTOR 13       /* cells per thread: 0 = auto (FP32: 1; otherwise groups of 8 bytes), or 1, 2, 4 (group <= 8 bytes, divides nx) */
#define LBM_P_BRICK 14        /* rows per brick of the device layout: 0 = auto (8; capped at ny).  Used only
                               * when every block of both step kernels holds a single row, otherwise the
                               * plain order (brick = ny).  Fixed once the state is initialised; reading it
                               * gives the height in use.  Results do not depend on it. */
#define LBM_P_ODD_ROWS 15     /* odd-step kernel: 0 = blocks of rows or row segments exchanging through LDS;
                               * 1 = (default) one wavefront per row walking it in 64-lane segments, for FP16/BF16
                               * and FP64 stores whose rows are longer than an odd-step block; 2 = walk rows whenever nx is a
                               * multiple of 64 cells
                               * per thread.  Results do not depend on it (statistics sums up to summation order). */
#define LBM_P_SPREAD 16       /* launch order: c in [5, 16] = chunks of 2^c tiles cycle through the bricks of the
                               * layout, so the wall rows (first and last brick; their Newton solves cost more)
                               * are spread over the whole launch; 0 = tiles in memory order; -1 (default) = 7
                               * for 2-byte stores, 0 otherwise.  Applies when every brick is whole and holds a
                               * whole number of chunks; reads back the value in use.  Results do not depend
                               * on it. */
#define LBM_P_ODD_BY_ROWS 17  /* read only: 1 if the odd step currently walks rows (k_odd_rows), 0 if it runs
                               * the block kernel, as decided by LBM_P_ODD_ROWS, the store, nx and the blocks */
#define LBM_P_COLLISION 18    /* 0 = BGK (default); 1 = MRT, the paper's collision (Sec. 3.1, after d'Humieres
                               * et al. 2002): the D3Q19 moment basis of that paper, equilibrium moments of the
                               * same second-order equilibrium (equal rates give BGK), the viscous stresses
                               * relaxed at 1/tau_e (Smagorinsky), the non-hydrodynamic moments at the rates
                               * below, the body force added as (I - S/2) M F in moment space */
#define LBM_P_MRT_S_E 19      /* MRT rate of the energy moment, in (0, 2); default 1.19 */
#define LBM_P_MRT_S_EPS 20    /* ... of the energy-square moment; default 1.4 */
#define LBM_P_MRT_S_Q 21      /* ... of the three heat-flux moments; default 1.2 */
#define LBM_P_MRT_S_PI 22     /* ... of the two fourth-order normal-stress moments; default 1.99, near the
                               * shear rate of a channel at tau0 -> 1/2.  A value fitted to Tables 2-3 (the
                               * paper states none): with d'Humieres' suggested 1.4, the documented
                               * alternative, the channel's mean profile falls well below the wall law */
#define LBM_P_MRT_S_M 23      /* ... of the three third-order moments; default 1.98 */
#define LBM_P_VD_APLUS 24     /* van Driest damping of the Smagorinsky constant (Sec. 3.1): Cs (1 - exp(-y+/A+))
                               * with y+ = d u_tau / nu0, d = min(y, ny - 1 - y) + y1; A+ >= 0, 0 = no damping
                               * (default); the paper's reference uses 26 */
#define LBM_P_VD_UTAU 25      /* friction velocity u_tau of that y+, >= 0; 0 (default) = sqrt(|Fx| ny / 2), the
                               * force-balance value of the channel */
#define LBM_P_WALL_NODES 26   /* wall placement, settable before the state is initialised: 0 (default) = link-wise
                               * walls halfway below row 0 and above row ny - 1, the WFB correction on the first
                               * fluid layer; 1 = wall nodes, the wall grid of Sec. 2.1-2.2 (Eq. 3, 4, 14 applied
                               * at the wall grid) as a lattice node one spacing below row 0 and above row
                               * ny - 1: the populations the first layer sends towards the wall reach the wall
                               * node of column x + e_b one step later, are reflected there (the boundary:
                               * bounce-back, mirror reflection or the WFB collision of Eq. 14 with tau_w of
                               * Eq. 15-17 from the first layer's density and velocity of that previous step)
                               * and stream into the fluid at the next step.  The wall records of lbm_wall_shear
                               * are then those of the next wall-node collision; lbm_wall_mass_change is not
                               * defined (LBM_E_STATE); state transfer restarts the wall nodes from the state
                               * (lbm_get_wall_nodes).  2 = the same wall nodes with tau_w from the first
                               * layer's density and velocity of the same step (the moments of what it gathers
                               * in that step), the wall records then those of the latest wall-node collision.
                               * Not for batches. */
#define LBM_P_XCD_CHUNK 27    /* with LBM_P_XCD_REMAP = 1: each of the 8 XCDs takes chunks of 2^c consecutive
                               * tiles in turn, c in [0, 12] (default 5; 0 = plain round robin).  Results do
                               * not depend on it.  Not for batches (their chunk is 2^5). */

typedef struct lbm_ctx lbm_ctx;

typedef struct {
    int32_t nx, ny, nz;
} lbm_grid;

/* Creates a channel context (no device memory yet).
 * g: grid with nx >= 1, ny >= 2, nz >= 1, nx * ny * nz < 2^31 and nx * ny < 2^29.
 * tau: molecular relaxation time, > 1/2; nu0 = (tau - 1/2) / 3 (BGK, Eq. 1).
 * Cs: Smagorinsky constant >= 0 (Sec. 3.1; the paper uses 0.1).
 * kappa, B: Spalding's law constants (Eq. 16; the paper uses 0.41 and 5.5).
 * Fx: body force density along x (the F_a of Eq. 1), any finite value.
 * On error returns LBM_E_ARG and leaves *out untouched.  Defaults: store F64,
 * boundary WFB, y1 = 1, Newton tol 1e-14 and cap 100, statistics off. */
int lbm_create(const lbm_grid* g, double tau, double Cs, double kappa, double B, double Fx, lbm_ctx** out);

/* Frees the context and its library-side device buffers (never the bound storage). */
void lbm_destroy(lbm_ctx* ctx);

int lbm_set_param(lbm_ctx* ctx, int key, double value);
int lbm_get_param(const lbm_ctx* ctx, int key, double* value);

/* Bytes of device storage the caller must bind: 19 * nx * ny * nz * sizeof(store). */
int lbm_required_bytes(const lbm_ctx* ctx, size_t* bytes);

/* Binds caller-owned device memory (e.g. a torch tensor) as the population
 * array.  dev_ptr must be 256-byte aligned and hold at least the required
 * bytes; the library never frees it.  The contents are undefined until an
 * lbm_init_* or lbm_set_state call.  Allocates the library's small side
 * buffers on the pointer's device. */
int lbm_bind_storage(lbm_ctx* ctx, void* dev_ptr, size_t bytes);

/* Sets the HIP stream (a hipStream_t, NULL = the default stream) on which all
 * of the context's device work is enqueued. */
int lbm_set_stream(lbm_ctx* ctx, void* hip_stream);

/* LBM_BB, LBM_WFB or LBM_FREESLIP; applies from the next step (and to the
 * observables of the current state). */
int lbm_set_boundary(lbm_ctx* ctx, int bc);

/* Initial state f = f_eq(1, u0) taken as post-collision populations:
 * u0 = U(y) (1 + d0, d1, d2) with U(y) = u_tau u+(y+), u+ from Spalding's law
 * (Eq. 16) at y+ = d u_tau / nu0, d = min(y, ny - 1 - y) + y1, and d_i uniform
 * in [-noise, noise) drawn by splitmix64 (Steele, Lea & Flood 2014) with
 * counter 3 c + i from state `seed`.  Resets the step count to 0. */
int lbm_init_spalding(lbm_ctx* ctx, double u_tau, double noise, uint64_t seed);

/* Initial state from given moments: f = f_eq(rho, u) of Eq. 1 (second-order
 * equilibrium) taken as post-collision populations, computed on the device
 * and rounded to the store format.  rho: ncells doubles, u: [3][ncells]
 * (u_x, u_y, u_z), both host arrays indexed c = x + nx (y + ny z).  Every
 * rho must be positive and every value finite (else LBM_E_ARG, nothing
 * written).  Resets the step count to 0.  Synchronises. */
int lbm_init_moments(lbm_ctx* ctx, const double* rho, const double* u);

/* Sets the state from host memory: h[a][c] = f*_a(c) - w_a, the post-collision
 * populations minus the weights, 19 * ncells doubles (rounded to the store
 * format).  Resets the step count to `steps`. Synchronises. */
int lbm_set_state(lbm_ctx* ctx, const double* h_host, int64_t steps);

/* Copies the state to host memory in the same canonical form as
 * lbm_set_state, whatever the internal layout.  cells == NULL: all cells,
 * out is [19][ncells]; otherwise out is [19][n] for the n listed cells.
 * Synchronises. */
int lbm_get_state(lbm_ctx* ctx, double* h_host);
int lbm_get_state_cells(lbm_ctx* ctx, int64_t n, const int64_t* cells, double* out);

/* Advances n >= 0 time steps.  Asynchronous; device-side failures surface at
 * the next synchronising call. */
int lbm_step(lbm_ctx* ctx, int64_t n);

/* Synchronises the stream and reports device-side failures: LBM_E_NONFINITE
 * or LBM_E_NEWTON, with the first failing step (1-based) in *first_bad_step
 * (may be NULL; -1 when none). */
int lbm_sync(lbm_ctx* ctx, int64_t* first_bad_step);

/* Steps done since the last initialisation. */
int lbm_steps_done(const lbm_ctx* ctx, int64_t* steps);

/* Observables of the current state: the gather and WFB correction the next
 * step would do, then rho and u = (sum e f + F/2) / rho (Eq. 2).  Host arrays
 * of ncells doubles each (any may be NULL), indexed by c.  Synchronises. */
int lbm_moments(lbm_ctx* ctx, double* rho, double* ux, double* uy, double* uz);
/* Same for n listed cells: out is [n][4] = rho, ux, uy, uz. */
int lbm_moments_cells(lbm_ctx* ctx, int64_t n, const int64_t* cells, double* out);

/* The same observables (Eq. 2 after the gather and WFB correction the next
 * step would make) written to caller-owned device memory on the context's
 * device: each non-NULL pointer receives ncells doubles indexed by c.  At
 * least one pointer must be given (else LBM_E_ARG).  Asynchronous on the
 * context's stream, like lbm_step; nothing is copied to the host. */
int lbm_moments_device(lbm_ctx* ctx, double* rho, double* ux, double* uy, double* uz);

/* Wall records of the current state, 2 * nx * nz doubles each (any may be
 * NULL), layout [w][z][x], w = 0 bottom, 1 top.  WFB: tau_x, tau_z (Eq. 15),
 * u_tau (Eq. 17) and the wall-parallel speed U fed to Spalding's law.  BB:
 * the wall force on the fluid by momentum exchange and u_tau = sqrt(|tau|/rho).
 * Free-slip: zeros and U.  Synchronises. */
int lbm_wall_shear(lbm_ctx* ctx, double* tau_x, double* tau_z, double* u_tau, double* U);

/* Distribution of the first-layer y+ over the wall cells (Fig. 7: the PDF of
 * y1+ normalised by its mean and standard deviation), computed on the device
 * from the current wall records: y+ = y1 u_tau / nu0 with nu0 = (tau0 - 1/2)/3.
 * mean_std[2] receives the mean and the population standard deviation of y+
 * (FP64, fixed summation order); counts[nbins + 2] the number of wall cells
 * whose z = (y+ - mean) / std falls below lo (counts[0]), in bin k of
 * [lo + k w, lo + (k + 1) w), w = (hi - lo) / nbins (counts[k + 1]), or at or
 * above hi (counts[nbins + 1]).  Host arrays, caller-owned; 1 <= nbins <= 2^20,
 * lo < hi, else LBM_E_ARG.  Synchronises. */
int lbm_wall_yplus_pdf(lbm_ctx* ctx, int32_t nbins, double lo, double hi, int64_t* counts, double* mean_std);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * distribution as lbm_wall_yplus_pdf, from the same kernels, with no
 * allocation.  counts[nbins + 2] and mean_std[2] are caller-owned DEVICE
 * memory on the context's device; the call only enqueues kernels on the
 * context's stream and returns (read the results after synchronising it).
 * The per-wall-cell friction velocities go to a fixed work area of 2^22
 * doubles (32 MiB) that the library holds on each device until the process
 * ends: grids with 2 nx nz > 2^22 wall cells get LBM_E_ARG.  Every call on a
 * device shares that work area, so calls that overlap on one device (other
 * streams, other contexts, other threads) race; calls in order on one stream
 * do not.  The step's failure flags are not checked (lbm_sync does that).
 * After a switch between bounce-back and mirror reflection the state may need
 * a re-layout that takes a buffer: then LBM_E_STATE until lbm_step or
 * lbm_wall_yplus_pdf has run. */
int lbm_wall_yplus_pdf_noalloc(lbm_ctx* ctx, int32_t nbins, double lo, double hi, int64_t* counts, double* mean_std);

/* Mass check of the wall correction (Appendix B, Eq. B-1): for every wall cell
 * the sum of the 19 populations after the WFB correction (Eq. 14) the next
 * step would make, minus the sum before it, as the step kernel computes them
 * (its own precision: FP64 for the FP64 store, FP32 otherwise; summed in
 * direction order over the deviations h_a = f_a - w_a the kernel holds, so the
 * weights cancel exactly).  In exact arithmetic it is zero; the value is the
 * round-off of the four corrected populations.  dsum and rho (either may be
 * NULL, not both) are host arrays of 2 * nx * nz doubles, layout [w][z][x]
 * (w = 0 bottom, 1 top); rho is the cell's density before the correction, so
 * that the mean population is rho / 19.  Zeros for bounce-back and free-slip
 * walls, whose reflections only permute.  Synchronises. */
int lbm_wall_mass_change(lbm_ctx* ctx, double* dsum, double* rho);

/* Wall-node state (LBM_P_WALL_NODES = 1 or 2, else LBM_E_STATE): fw [2][5][nz][nx]
 * receives, as h = f - w, the populations each wall node sends into the fluid
 * at the next step (walls w = 0 bottom, 1 top; directions 3, 7, 11, 14, 17
 * at the bottom and their mirror images 4, 13, 18, 8, 12 at the top); rec
 * [2][nz][nx][4] the first layer's density, u_x, u_z and friction velocity of
 * the latest step, from which the next wall-node collision takes its stress.
 * After a state is set or initialised the wall nodes start from it: the
 * record from the plain moments of the first layer's post-collision
 * populations, and one wall-node collision of them.  Either pointer may be
 * NULL, not both.  Synchronises. */
int lbm_get_wall_nodes(lbm_ctx* ctx, double* fw, double* rec);

/* Plane statistics (Sec. 3.1 time and plane averages, Fig. 6 moments),
 * accumulated in FP64 on sampled steps from the velocity each sampled step
 * computes.  lbm_stats_sums: out[y][8] = sums of ux, uy, uz, ux^2, uy^2, uz^2,
 * ux uy and the number of cell samples.  lbm_stats_get: out[y][8] = <ux>,
 * <uy>, <uz>, <ux'^2>, <uy'^2>, <uz'^2>, <ux'uy'>, cell samples.  Both
 * synchronise; nsamples (may be NULL) receives the number of sampled steps. */
int lbm_stats_reset(lbm_ctx* ctx);
int lbm_stats_sums(lbm_ctx* ctx, double* out, int64_t* nsamples);
int lbm_stats_get(lbm_ctx* ctx, double* out, int64_t* nsamples);

/* Picks the launch shapes of the step kernels by timing them on the bound
 * storage: the block sizes of the odd and even kernels (64, 128, 256, 512),
 * the cells per thread (1, 2, 4 where the store and nx allow), the rows per
 * brick of the layout (4, 8, 16, 32), the launch order (LBM_P_SPREAD: memory
 * order or chunks of 2^5, 2^7, 2^9 tiles), whether the odd step walks
 * rows (LBM_P_ODD_ROWS) and the XCD chunk (LBM_P_XCD_CHUNK: 2^5, 2^7, 2^9
 * tiles).  Coordinate descent from the context's current
 * shapes, one setting at a time, each candidate timed over `steps` steps
 * (>= 2) after one warm-up pair; a change is kept only when it is more than
 * 1 % faster (the odd-step settings decided by the odd kernel's time, the even
 * block size by the even kernel's, the rest by both).  The result is kept for the
 * life of the process per (device, grid, store, boundary, collision, wall
 * placement): a later call with the same key applies it without timing.
 * None of these settings changes a result bit.  Valid only before the state
 * is initialised (it writes the initial profile the body force implies);
 * afterwards the state is undefined until lbm_init_* / lbm_set_state.
 * Synchronises.  choice (may be NULL) receives eight values: the odd and even
 * block sizes, the cells per thread, the rows per brick in use, the launch
 * order's chunk log2 (0: memory order), 1 if the odd step walks rows, 1 if
 * the result came from the cache, and the XCD chunk log2. */
int lbm_autotune(lbm_ctx* ctx, int steps, int32_t* choice);

/* Spalding's law inverted on the host (Eq. 16): u+ for a given y+ >= 0. */
int lbm_spalding_uplus(double yplus, double kappa, double B, double* uplus);

/* The device wall-function solve on n host values of the wall-parallel speed
 * U: u_tau[i] (-1 on an iteration-cap failure) and iterations[i].  Uses the
 * same device code as the step.  Synchronises the default stream. */
int lbm_device_wall_utau(int32_t n, const double* U, double y1, double nu, double kappa, double B, double tol,
                         int32_t maxit, double* u_tau, int32_t* iterations);

/* Round trip of n host floats through the store format's device codec, the
 * same conversion code the step kernels use (narrowing rounds to nearest,
 * ties to even): out[i] = decode(encode(in[i])).  Synchronises. */
int lbm_codec_roundtrip(int store, int64_t n, const float* in, float* out);

/* Streams `bytes` (a multiple of 16) from src to dst on the device with a
 * plain copy kernel (16-byte non-temporal accesses, one 16 KB chunk per block,
 * blocks handed to the XCDs in chunks like the step kernels'); a probe of the
 * achievable HBM bandwidth.  dst may equal src (an in-place pass, the AA
 * step's access form); otherwise the ranges must not overlap.  Asynchronous
 * on hip_stream. */
int lbm_copy_probe(void* dst, const void* src, size_t bytes, void* hip_stream);

/* ------------------------------------------------------------------------
 * Batched ensembles: many independent channels (own grid, tau, Cs, Fx and
 * boundary each) advanced together, one launch per time step over the tiles
 * of every instance (and HIP-graph chunks of such launches).  Instances share
 * the store format, block sizes, cells per thread, stream and one pooled
 * storage buffer; instance i's populations start at a 256-byte aligned
 * offset in the order of creation.  Each instance evolves exactly as the same
 * channel stepped alone with the same launch shape.  Plane statistics are not
 * sampled in batches.
 * ------------------------------------------------------------------------ */
typedef struct lbm_batch lbm_batch;

/* n >= 1 instances: grids[i], tau[i], Cs[i], Fx[i] and bc[i] (LBM_BB, LBM_WFB
 * or LBM_FREESLIP) as for lbm_create; kappa and B shared.  LBM_E_ARG names
 * the first bad instance in lbm_batch_last_error(NULL); *out untouched on error. */
int lbm_batch_create(int32_t n, const lbm_grid* grids, const double* tau, const double* Cs, const double* Fx,
                     const int32_t* bc, double kappa, double B, lbm_batch** out);
void lbm_batch_destroy(lbm_batch* batch);
/* Keys LBM_P_STORE (before binding), LBM_P_TILE_ODD, LBM_P_TILE_EVEN,
 * LBM_P_VECTOR (0 = automatic: FP32 one cell per thread, otherwise the widest group every instance allows), LBM_P_XCD_REMAP,
 * LBM_P_GRAPH_STEPS, LBM_P_SPREAD, LBM_P_ODD_ROWS (walks rows only if every instance's rows
 * qualify), and LBM_P_Y1 / LBM_P_NEWTON_TOL / LBM_P_NEWTON_MAXIT /
 * LBM_P_BRICK (before initialisation) applied to every instance.  Block
 * sizes and cells per thread that an initialised instance's layout cannot
 * run with give LBM_E_STATE. */
int lbm_batch_set_param(lbm_batch* batch, int key, double value);
/* Sum over instances of their required bytes, each rounded up to 256. */
int lbm_batch_required_bytes(const lbm_batch* batch, size_t* bytes);
/* Caller-owned device memory, 256-byte aligned, at least the required bytes. */
int lbm_batch_bind_storage(lbm_batch* batch, void* dev_ptr, size_t bytes);
int lbm_batch_set_stream(lbm_batch* batch, void* hip_stream);
/* lbm_init_spalding for every instance: u_tau[i], seeds[i], shared noise. */
int lbm_batch_init_spalding(lbm_batch* batch, const double* u_tau, double noise, const uint64_t* seeds);
/* Advances every instance n >= 0 steps.  Asynchronous. */
int lbm_batch_step(lbm_batch* batch, int64_t n);
/* Synchronises; reports the first instance (and its first step) whose device
 * status is set, else LBM_OK.  Either pointer may be NULL. */
int lbm_batch_sync(lbm_batch* batch, int64_t* first_bad_step, int32_t* first_bad_instance);
/* Instance i as a context for observation (lbm_moments, lbm_wall_shear,
 * lbm_get_state, ...); stepping, setting state or parameters through it
 * returns LBM_E_STATE.  Owned by the batch.  NULL when i is out of range. */
lbm_ctx* lbm_batch_instance(lbm_batch* batch, int32_t i);
/* Picks the launch shapes of the batched launch by timing them (valid only
 * before the state is initialised, as lbm_autotune): every cells-per-thread
 * width the instances allow with every block size (64-512 threads; the odd
 * and even kernels timed apart, the width shared), then the odd step's row
 * walk switched off or forced (LBM_P_ODD_ROWS 0, 2), kept when more than 1 %
 * faster.  tiles (may be NULL) receives the odd and even block sizes and the
 * cells per thread. */
int lbm_batch_autotune(lbm_batch* batch, int steps, int32_t* tiles);
const char* lbm_batch_last_error(const lbm_batch* batch);

const char* lbm_status_str(int status);
/* Text of the last error of ctx (valid until the next call on ctx), or of the
 * last error of a call without a context when ctx is NULL. */
const char* lbm_last_error(const lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBMWF_H */
