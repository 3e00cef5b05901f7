// C ABI of the WFB LBM-LES channel library: contexts, argument checking,
// storage binding, launch sequencing (AA parity, HIP graph chunks),
// observation, statistics and the block-size autotuner.  Declared in
// include/lbmwf.h; the device code lives in lbm_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "lbm_internal.h"
#include "lbmwf.h"
#include "store.h"

using namespace lbmwf;

namespace {

thread_local std::string g_err;  // errors of calls without a context

struct GraphKey {
    int layout_s, len, stats_every;
    long long phase;
    bool operator<(const GraphKey& o) const
    {
        return std::tie(layout_s, len, stats_every, phase) < std::tie(o.layout_s, o.len, o.stats_every, o.phase);
    }
};

}  // namespace

// Work area of lbm_wall_yplus_pdf_noalloc: the friction velocity of each wall
// cell (2 nx nz of them, at most kScratchWallCells = 2^22, 32 MiB).  Every
// device the library runs on holds its own copy until the process ends; host
// code reaches it only through the address scratch_address() looked up on that
// device, never through this name.
constexpr long long kScratchWallCells = 1ll << 22;
static __device__ __align__(256) double scratch[kScratchWallCells];

namespace {

constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
bool g_scratch_done[kMaxDevices];

// Device address of the work area on device dev, which must be current; the
// first call per device looks it up (hipGetSymbolAddress) and keeps the result.
hipError_t scratch_address(int dev, double** out)
{
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[dev]) {
        void* p = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? (double*)p : nullptr;
        g_scratch_done[dev] = true;
    }
    *out = g_scratch_ptr[dev];
    return g_scratch_err[dev];
}

// Device of a device-memory pointer, or -1 (host or unknown memory).  A failed
// query leaves no error behind for the next launch check to pick up.
int device_of(const void* p)
{
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    return attr.type == hipMemoryTypeDevice ? attr.device : -1;
}

}  // namespace

struct lbm_ctx {
    int nx = 0, ny = 0, nz = 0;
    long long n = 0;
    double tau0 = 0, cs = 0, kappa = 0, bconst = 0, fx = 0;
    double y1 = 1.0, newton_tol = 1e-14;
    int newton_maxit = 100;
    int store = kStoreF64;
    int bc = kWFB;
    int stats_every = 0;
    int tile_odd = 256, tile_even = 256, xcd_remap = 1, graph_steps = 32;
    int xcd_chunk = kXcdChunkLog2;   // log2 of the consecutive tiles each XCD takes in turn (LBM_P_XCD_CHUNK)
    int vw_req = 0;              // cells per thread requested; 0 = automatic (auto_vector_width)
    int brick_req = 0;           // rows per brick of the population layout requested; 0 = automatic
    int brick = 0;               // rows per brick in use; fixed while the state is initialised
    int odd_rows = 1;            // odd step by rows: 0 never, 1 when rows are longer than a block, 2 whenever possible
    int coll = kBGK;             // collision: kBGK or kMRT
    // MRT rates e, epsilon, q, pi, m: d'Humieres et al. (2002) for e, epsilon, q, m; the fourth-order
    // normal stresses near the shear rate, a value fitted so that the wall-law runs match Tables 2-3
    // (the paper states none; the reference suggests 1.4)
    double mrt_s[5] = {1.19, 1.4, 1.2, 1.99, 1.98};
    double vd_aplus = 0.0;       // van Driest A+; 0 = no damping
    double vd_utau = 0.0;        // friction velocity of the damping's y+; 0 = sqrt(|Fx| ny / 2)
    int spread = -1;             // launch order: log2 of the tile chunks that cycle through the bricks; 0 = memory
                                 // order; -1 = by store format (spread_log2)
    int wall_nodes = 0;          // 1: wall nodes one spacing outside the first and last layer (fixed once initialised)
    void* dwn = nullptr;         // wall-node rings (wn_index) and first-layer records
    double* dwn_rec = nullptr;

    void* h = nullptr;
    size_t bytes = 0;
    int dev = -1;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;

    DevFlags* dflags = nullptr;
    double* dacc = nullptr;      // [ny][8]
    double* dprof = nullptr;     // [ny]
    double* dpart = nullptr;     // [max tiles][7]
    size_t part_cap = 0;         // tiles
    double* dtmp = nullptr;      // relayout scratch, [2 nx nz][5]
    double* dcs2 = nullptr;      // [ny] 18 Cs^2 with the van Driest damping
    std::vector<double> hcs2;    // its host copy
    bool cs2_dirty = true;

    bool initialized = false;
    long long steps = 0;
    int layout_s = 0;            // 1 after an odd number of steps
    int layout_spec = 0;         // reflections stored in layout S were mirror images
    long long nsamples = 0;

    std::map<GraphKey, hipGraphExec_t> graphs;
    std::string err;
    bool batch_member = false;   // stepped by its batch; observation only
};

namespace {

int fail(lbm_ctx* ctx, int code, const std::string& msg)
{
    if (ctx) ctx->err = msg;
    else g_err = msg;
    return code;
}

// Error text without allocation failures escaping: an exception never
// crosses the C ABI, so the guard below reports it with this.
int fail_nothrow(lbm_ctx* ctx, int code, const char* msg) noexcept
{
    try {
        if (ctx) ctx->err = msg;
        else g_err = msg;
    } catch (...) {
    }
    return code;
}

// Runs the body of an entry point; a C++ exception (a host allocation
// failure in a container or string) becomes a status code.
template <typename F>
int guard(lbm_ctx* ctx, F&& body) noexcept
{
    try {
        return body();
    } catch (const std::bad_alloc&) {
        return fail_nothrow(ctx, LBM_E_OOM, "host memory allocation failed");
    } catch (...) {
        return fail_nothrow(ctx, LBM_E_STATE, "internal error (exception)");
    }
}

#define LBM_HIP(ctx, call)                                                                      \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail((ctx), LBM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (dev >= 0 && hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Cells per thread when none is requested: one for FP32, whose odd step then
// reads its x-shifted neighbours directly instead of exchanging groups through
// LDS (on 2048-cell rows 29.9 ms against 31.1 ms at two cells per thread;
// the 64-channel FP32 ensemble's step pair 8 % faster);
// otherwise the widest 8-byte group that divides nx (FP16/BF16: four cells).
int auto_vector_width(int store, int nx)
{
    return store == LBM_STORE_F32 ? 1 : step_vector_width(store, nx);
}

int vector_width(const lbm_ctx* c)
{
    if (c->vw_req > 0 && step_vector_width_ok(c->store, c->nx, c->vw_req)) return c->vw_req;
    return auto_vector_width(c->store, c->nx);
}

// row segments (x segments times rows) of the statistics partial sums
long long segments_for(const lbm_ctx* c, int tile)
{
    StepArgs g{};
    step_geometry(c->nx, c->ny, c->nz, tile, vector_width(c), c->ny, g);
    return (long long)g.ntx * c->ny * c->nz;
}

int rows_per_block(const lbm_ctx* c, int tile, int vw)
{
    StepArgs g{};
    step_geometry(c->nx, c->ny, c->nz, tile, vw, c->ny, g);
    return g.rpb;
}

// Rows per brick for the current launch shapes: bricks of 8 rows (or the
// requested height) when every block holds a single row, else the plain
// [z][y][x] order (one brick of ny rows).
constexpr int kAutoBrick = 8;
int brick_for_tiles(const lbm_ctx* c)
{
    const int vw = vector_width(c);
    if (rows_per_block(c, c->tile_odd, vw) > 1 || rows_per_block(c, c->tile_even, vw) > 1) return c->ny;
    return std::min(c->brick_req > 0 ? c->brick_req : kAutoBrick, c->ny);
}

// the layout of the current state (fixed once it is initialised)
int brick_rows(const lbm_ctx* c) { return c->initialized ? c->brick : brick_for_tiles(c); }

// launch shapes that can run on the initialised state's layout
bool shapes_fit_layout(const lbm_ctx* c)
{
    if (!c->initialized) return true;
    const int vw = vector_width(c);
    return brick_ok(c->ny, c->brick, rows_per_block(c, c->tile_odd, vw)) &&
           brick_ok(c->ny, c->brick, rows_per_block(c, c->tile_even, vw));
}

bool tile_ok(int t) { return t == 64 || t == 128 || t == 256 || t == 512; }

// Destroys the cached graph executables; a launch of one may still be
// running (lbm_step is asynchronous), so the stream is drained first.
void drop_graphs(lbm_ctx* c)
{
    if (c->graphs.empty()) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

// The tuners' three timing events, destroyed on every way out of the tuner
// (error returns and host exceptions included).
struct TimingEvents {
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    bool create()
    {
        for (auto& e : ev)
            if (hipEventCreate(&e) != hipSuccess) {
                e = nullptr;
                return false;
            }
        return true;
    }
    ~TimingEvents()
    {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

// Whether the odd step walks rows (one wavefront per row) for these shapes.
// Automatic (mode 1): for 2-byte and 8-byte stores whose rows are longer than
// an odd-step block.  On the 2048 x 512 x 1024 channel the walk beat row
// segments exchanging through LDS by 5 % in FP16; in FP64 it runs as fast as
// the blocks' direct shifted loads (52.3 against 52.4 ms) and writes every
// 128-byte line once, where the blocks' shifted segment-edge stores wrote
// 0.6 % more.  FP32 and short rows keep the blocks (as fast or faster).
bool odd_by_rows(const lbm_ctx* c, int mode)
{
    const int vw = vector_width(c);
    if (mode == 0 || c->wall_nodes || !rows_ok(c->nx, vw)) return false;
    const int bytes = store_bytes(c->store);
    return mode == 2 || ((bytes == 2 || bytes == 8) && c->nx / vw > c->tile_odd);
}

// Chunk size of the brick-spreading launch order (LBM_P_SPREAD = -1): the
// wall rows' Newton solves weigh most against the short steps of 2-byte
// stores, which spread in chunks of 128 tiles (measured on MI355X: 6-9 %
// faster steps of the 512x128x256 channel); 4- and 8-byte stores keep the
// memory order (spreading them cost 1-5 %).
constexpr int kSpreadLog2Short = 7;
int spread_log2(const lbm_ctx* c)
{
    if (c->spread >= 0) return c->spread;
    return store_bytes(c->store) == 2 ? kSpreadLog2Short : 0;
}

StepArgs step_args(const lbm_ctx* c, bool odd, int rows_mode)
{
    StepArgs a{};
    a.h = c->h;
    a.n = c->n;
    a.nx = c->nx;
    a.ny = c->ny;
    a.nz = c->nz;
    if (odd && odd_by_rows(c, rows_mode))
        step_geometry_rows(c->nx, c->ny, c->nz, c->tile_odd, vector_width(c), brick_rows(c), a);
    else
        step_geometry(c->nx, c->ny, c->nz, odd ? c->tile_odd : c->tile_even, vector_width(c), brick_rows(c), a);
    a.tile_begin = 0;
    a.bc = c->bc;
    a.xcd_remap = c->xcd_remap ? c->xcd_chunk + 1 : 0;
    set_spread(a, spread_log2(c));
    a.newton_maxit = c->newton_maxit;
    a.tau0 = c->tau0;
    a.cs2_18 = 18.0 * c->cs * c->cs;
    a.cs2_row = (c->vd_aplus > 0.0) ? c->dcs2 : nullptr;
    a.coll = c->coll;
    for (int i = 0; i < 5; ++i) a.mrt_s[i] = c->mrt_s[i];
    a.fx = c->fx;
    a.y1 = c->y1;
    a.nu0 = (c->tau0 - 0.5) / 3.0;
    a.kappa = c->kappa;
    a.bconst = c->bconst;
    a.ekb = std::exp(-c->kappa * c->bconst);
    a.newton_tol = c->newton_tol;
    a.flags = c->dflags;
    a.partials = nullptr;
    a.wall_nodes = c->wall_nodes;
    a.wn = c->dwn;
    a.wn_rec = c->dwn_rec;
    return a;
}

ObsArgs obs_args(const lbm_ctx* c)
{
    ObsArgs a{};
    a.h = c->h;
    a.n = c->n;
    a.nx = c->nx;
    a.ny = c->ny;
    a.nz = c->nz;
    a.brick = brick_rows(c);
    a.layout_s = c->layout_s;
    a.bc = c->bc;
    a.layout_spec = c->layout_spec;
    a.newton_maxit = c->newton_maxit;
    a.fx = c->fx;
    a.y1 = c->y1;
    a.nu0 = (c->tau0 - 0.5) / 3.0;
    a.kappa = c->kappa;
    a.bconst = c->bconst;
    a.ekb = std::exp(-c->kappa * c->bconst);
    a.newton_tol = c->newton_tol;
    a.wall_nodes = c->wall_nodes;
    a.wn = c->dwn;
    a.wn_rec = c->dwn_rec;
    return a;
}

bool sampled(const lbm_ctx* c, long long t) { return c->stats_every > 0 && t % c->stats_every == 0; }

// Enqueues `len` steps starting after step t0 from layout `layout_s` on stream s.
// Pure with respect to the context's bookkeeping (used for eager launches and
// for graph capture).
hipError_t enqueue_steps(const lbm_ctx* c, hipStream_t s, int layout_s, long long t0, long long len)
{
    const StepArgs ao = step_args(c, true, c->odd_rows), ae = step_args(c, false, c->odd_rows);
    for (long long i = 0; i < len; ++i) {
        const long long t = t0 + 1 + i;
        const bool odd = (layout_s == 0);
        const bool st = sampled(c, t);
        StepArgs a = odd ? ao : ae;
        if (st) a.partials = c->dpart;
        hipError_t e = launch_step(c->store, odd, c->bc, a, s);
        if (e != hipSuccess) return e;
        if (st) {
            e = launch_stats_reduce(c->dpart, a.ntx, c->ny, c->nz, c->nx, c->dacc, s);
            if (e != hipSuccess) return e;
        }
        layout_s ^= 1;
    }
    return hipSuccess;
}

void advance_bookkeeping(lbm_ctx* c, long long len)
{
    for (long long i = 0; i < len; ++i) {
        const long long t = c->steps + 1;
        if (c->layout_s == 0) c->layout_spec = (c->bc != kBB);
        if (sampled(c, t)) c->nsamples += 1;
        c->layout_s ^= 1;
        c->steps = t;
    }
}

int ensure_partials(lbm_ctx* c)
{
    if (c->stats_every <= 0) return LBM_OK;
    const size_t need = (size_t)std::max(segments_for(c, c->tile_odd), segments_for(c, c->tile_even));
    if (need <= c->part_cap) return LBM_OK;
    drop_graphs(c);
    if (c->dpart) (void)hipFree(c->dpart);
    c->dpart = nullptr;
    c->part_cap = 0;
    LBM_HIP(c, hipMalloc((void**)&c->dpart, need * 7 * sizeof(double)));
    c->part_cap = need;
    return LBM_OK;
}

int reset_flags(lbm_ctx* c)
{
    DevFlags f{};
    f.status = 0;
    f.max_newton_iters = 0;
    f.first_bad = ~0ull;
    f.cnt[0] = f.cnt[1] = c->steps + 1;
    LBM_HIP(c, hipMemcpyAsync(c->dflags, &f, sizeof(f), hipMemcpyHostToDevice, c->stream));
    LBM_HIP(c, hipStreamSynchronize(c->stream));  // f lives on the host stack
    return LBM_OK;
}

int read_flags(lbm_ctx* c, DevFlags* f)
{
    LBM_HIP(c, hipStreamSynchronize(c->stream));
    LBM_HIP(c, hipMemcpy(f, c->dflags, sizeof(DevFlags), hipMemcpyDeviceToHost));
    return LBM_OK;
}

int status_of(const DevFlags& f)
{
    if (f.status & 1) return LBM_E_NONFINITE;
    if (f.status & 2) return LBM_E_NEWTON;
    return LBM_OK;
}

// Synchronise and report any device-side failure.
int sync_check(lbm_ctx* c)
{
    DevFlags f;
    int st = read_flags(c, &f);
    if (st != LBM_OK) return st;
    st = status_of(f);
    if (st != LBM_OK)
        return fail(c, st, std::string(lbm_status_str(st)) + " at step " + std::to_string((long long)f.first_bad));
    return LBM_OK;
}

int check_ready(lbm_ctx* c)
{
    if (!c) return fail(nullptr, LBM_E_ARG, "null context");
    if (!c->h) return fail(c, LBM_E_STATE, "no storage bound");
    if (!c->initialized) return fail(c, LBM_E_STATE, "state not initialised");
    return LBM_OK;
}

// Moves the wall-crossing populations of a streamed layout when the boundary
// switched between bounce-back and mirror reflection (halfway walls only:
// with wall nodes the reflection happens in the wall-node collision).
// Whether the state must be re-laid out before it is read: a streamed layout
// whose wall reflections were made by the other rule than the current boundary's.
bool layout_stale(const lbm_ctx* c)
{
    return c->initialized && c->layout_s && !c->wall_nodes && (int)(c->bc != kBB) != c->layout_spec;
}

int fix_layout(lbm_ctx* c)
{
    if (!layout_stale(c)) return LBM_OK;
    const int want = (c->bc != kBB);
    if (!c->dtmp) LBM_HIP(c, hipMalloc((void**)&c->dtmp, (size_t)2 * c->nx * c->nz * 5 * sizeof(double)));
    LBM_HIP(c, launch_relayout(c->store, c->h, c->n, c->nx, c->ny, c->nz, c->brick, c->layout_spec, want, c->dtmp,
                               c->stream));
    c->layout_spec = want;
    return LBM_OK;
}

// Wall-node rings and records (allocated with the first initialisation in
// wall-node mode; 4 rings of 10 nx nz elements, 2 nx nz records of 4 doubles).
int ensure_wall_nodes(lbm_ctx* c)
{
    if (!c->wall_nodes || c->dwn) return LBM_OK;
    const size_t ring = (size_t)10 * c->nx * c->nz * (size_t)store_bytes(c->store);
    LBM_HIP(c, hipMalloc(&c->dwn, 4 * ring));
    LBM_HIP(c, hipMalloc((void**)&c->dwn_rec, (size_t)2 * c->nx * c->nz * 4 * sizeof(double)));
    return LBM_OK;
}

// After a state set from outside (layout P): the wall nodes start from it.
int start_wall_nodes(lbm_ctx* c)
{
    if (!c->wall_nodes) return LBM_OK;
    int st = ensure_wall_nodes(c);
    if (st != LBM_OK) return st;
    LBM_HIP(c, launch_node_start(c->store, step_args(c, false, 0), c->stream));
    return LBM_OK;
}

// u+ of Spalding's law (Eq. 16) at y+: Newton on Sp(p) - y+ = 0 from a start
// to the right of the root (Sp(p) >= p, and the log-law estimate plus a margin
// when it is also to the right), where Newton on the increasing convex
// function converges monotonically.
double spalding_uplus_host(double yp, double kappa, double b)
{
    if (!(yp > 0.0)) return 0.0;
    const double ekb = std::exp(-kappa * b);
    auto sp = [&](double p) {
        const double k = kappa * p;
        return p + ekb * (std::expm1(k) - k - 0.5 * k * k - k * k * k / 6.0);
    };
    double p = yp;
    const double alt = b + std::log1p(yp) / kappa + 2.0;
    if (alt < p && sp(alt) >= yp) p = alt;
    for (int it = 0; it < 400; ++it) {
        const double k = kappa * p;
        const double g = sp(p) - yp;
        const double dg = 1.0 + kappa * ekb * (std::expm1(k) - k - 0.5 * k * k);
        const double pn = p - g / dg;
        if (!(pn < p)) break;  // monotone decrease has stopped: converged to round-off
        p = pn;
    }
    return p;
}

}  // namespace

// ===================================================================== API

extern "C" {

const char* lbm_status_str(int s)
{
    switch (s) {
        case LBM_OK: return "ok";
        case LBM_E_ARG: return "invalid argument";
        case LBM_E_STATE: return "invalid state";
        case LBM_E_OOM: return "out of memory";
        case LBM_E_DEVICE: return "device error";
        case LBM_E_NONFINITE: return "non-finite density";
        case LBM_E_NEWTON: return "wall-function Newton solve did not converge";
    }
    return "unknown status";
}

const char* lbm_last_error(const lbm_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

int lbm_create(const lbm_grid* g, double tau, double Cs, double kappa, double B, double Fx, lbm_ctx** out)
{
    return guard(nullptr, [&]() -> int {
        if (!g || !out) return fail(nullptr, LBM_E_ARG, "null argument");
        if (g->nx < 1 || g->ny < 2 || g->nz < 1) return fail(nullptr, LBM_E_ARG, "grid needs nx >= 1, ny >= 2, nz >= 1");
        const long long n = (long long)g->nx * g->ny * g->nz;
        if (n >= (1ll << 31)) return fail(nullptr, LBM_E_ARG, "grid too large: nx * ny * nz must be below 2^31");
        if ((long long)g->nx * g->ny >= (1ll << 29))
            return fail(nullptr, LBM_E_ARG, "grid too large: nx * ny must be below 2^29 (32-bit offsets within a z-plane)");
        if (!std::isfinite(tau) || !(tau > 0.5)) return fail(nullptr, LBM_E_ARG, "tau must be finite and > 1/2");
        if (!std::isfinite(Cs) || !(Cs >= 0.0)) return fail(nullptr, LBM_E_ARG, "Cs must be finite and >= 0");
        if (!std::isfinite(kappa) || !(kappa > 0.0)) return fail(nullptr, LBM_E_ARG, "kappa must be finite and > 0");
        if (!std::isfinite(B) || !std::isfinite(Fx)) return fail(nullptr, LBM_E_ARG, "B and Fx must be finite");
        lbm_ctx* c = new (std::nothrow) lbm_ctx();
        if (!c) return fail(nullptr, LBM_E_OOM, "context allocation failed");
        c->nx = g->nx;
        c->ny = g->ny;
        c->nz = g->nz;
        c->n = n;
        c->tau0 = tau;
        c->cs = Cs;
        c->kappa = kappa;
        c->bconst = B;
        c->fx = Fx;
        *out = c;
        return LBM_OK;
    });
}

void lbm_destroy(lbm_ctx* c)
{
    if (!c) return;
    DeviceGuard dg(c->dev);
    if (c->stream || c->dflags) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->dflags) (void)hipFree(c->dflags);
    if (c->dacc) (void)hipFree(c->dacc);
    if (c->dprof) (void)hipFree(c->dprof);
    if (c->dpart) (void)hipFree(c->dpart);
    if (c->dtmp) (void)hipFree(c->dtmp);
    if (c->dcs2) (void)hipFree(c->dcs2);
    if (c->dwn) (void)hipFree(c->dwn);
    if (c->dwn_rec) (void)hipFree(c->dwn_rec);
    delete c;
}

int lbm_set_param(lbm_ctx* c, int key, double v)
{
    return guard(c, [&]() -> int {
        if (!c) return fail(nullptr, LBM_E_ARG, "null context");
        if (c->batch_member) return fail(c, LBM_E_STATE, "a batch instance's parameters are set through its batch");
        if (!std::isfinite(v)) return fail(c, LBM_E_ARG, "parameter value must be finite");
        const bool integral = (v == std::floor(v));
        switch (key) {
            case LBM_P_Y1:
                if (!(v > 0.0)) return fail(c, LBM_E_ARG, "y1 must be > 0");
                c->y1 = v;
                break;
            case LBM_P_NEWTON_TOL:
                if (!(v > 0.0)) return fail(c, LBM_E_ARG, "Newton tolerance must be > 0");
                c->newton_tol = v;
                break;
            case LBM_P_NEWTON_MAXIT:
                if (!integral || v < 1 || v > 10000) return fail(c, LBM_E_ARG, "Newton cap must be an integer in [1, 10000]");
                c->newton_maxit = (int)v;
                break;
            case LBM_P_STATS_EVERY:
                if (!integral || v < 0 || v > 1e9) return fail(c, LBM_E_ARG, "statistics interval must be an integer >= 0");
                c->stats_every = (int)v;
                break;
            case LBM_P_STORE:
                if (c->h) return fail(c, LBM_E_STATE, "the store format is fixed once storage is bound");
                if (!integral || v < 0 || v > 3) return fail(c, LBM_E_ARG, "store must be 0..3");
                c->store = (int)v;
                return LBM_OK;
            case LBM_P_TILE_ODD:
            case LBM_P_TILE_EVEN: {
                if (!integral || !tile_ok((int)v)) return fail(c, LBM_E_ARG, "tile must be 64, 128, 256 or 512");
                int& tile = (key == LBM_P_TILE_ODD ? c->tile_odd : c->tile_even);
                const int old = tile;
                tile = (int)v;
                if (!shapes_fit_layout(c)) {
                    tile = old;
                    return fail(c, LBM_E_STATE, "blocks of several rows need the plain layout; this state was initialised "
                                                "with bricks of " + std::to_string(c->brick) + " rows");
                }
                break;
            }
            case LBM_P_XCD_REMAP:
                if (v != 0.0 && v != 1.0) return fail(c, LBM_E_ARG, "XCD remap is 0 or 1");
                c->xcd_remap = (int)v;
                break;
            case LBM_P_XCD_CHUNK:
                if (!integral || v < 0 || v > 12) return fail(c, LBM_E_ARG, "XCD chunk is a tile-count log2 in [0, 12]");
                c->xcd_chunk = (int)v;
                break;
            case LBM_P_VECTOR: {
                if (!integral || (v != 0.0 && !step_vector_width_ok(c->store, c->nx, (int)v)))
                    return fail(c, LBM_E_ARG, "cells per thread must be 0 (auto) or 1, 2, 4 with groups of at most 8 bytes dividing nx");
                const int old = c->vw_req;
                c->vw_req = (int)v;
                if (!shapes_fit_layout(c)) {
                    c->vw_req = old;
                    return fail(c, LBM_E_STATE, "blocks of several rows need the plain layout; this state was initialised "
                                                "with bricks of " + std::to_string(c->brick) + " rows");
                }
                break;
            }
            case LBM_P_ODD_ROWS:
                if (!integral || v < 0 || v > 2) return fail(c, LBM_E_ARG, "odd-step mode must be 0, 1 or 2");
                c->odd_rows = (int)v;
                break;
            case LBM_P_SPREAD:
                if (!integral || v < -1 || v > 16 || (v > 0 && v < kXcdChunkLog2))
                    return fail(c, LBM_E_ARG, "brick spreading is -1 (by store), 0 (off) or a chunk log2 in [5, 16]");
                c->spread = (int)v;
                break;
            case LBM_P_BRICK:
                if (c->initialized) return fail(c, LBM_E_STATE, "the population layout is fixed once the state is initialised");
                if (!integral || v < 0 || v > (1 << 30)) return fail(c, LBM_E_ARG, "rows per brick must be an integer >= 0");
                c->brick_req = (int)v;
                break;
            case LBM_P_GRAPH_STEPS:
                if (!integral || v < 0 || v > 4096) return fail(c, LBM_E_ARG, "graph chunk must be an integer in [0, 4096]");
                c->graph_steps = (int)v;
                break;
            case LBM_P_FX:
                c->fx = v;
                break;
            case LBM_P_CS:
                if (!(v >= 0.0)) return fail(c, LBM_E_ARG, "Cs must be >= 0");
                c->cs = v;
                break;
            case LBM_P_COLLISION:
                if (v != kBGK && v != kMRT) return fail(c, LBM_E_ARG, "collision is 0 (BGK) or 1 (MRT)");
                c->coll = (int)v;
                break;
            case LBM_P_MRT_S_E:
            case LBM_P_MRT_S_EPS:
            case LBM_P_MRT_S_Q:
            case LBM_P_MRT_S_PI:
            case LBM_P_MRT_S_M:
                if (!(v > 0.0 && v < 2.0)) return fail(c, LBM_E_ARG, "MRT rates must lie in (0, 2)");
                c->mrt_s[key - LBM_P_MRT_S_E] = v;
                break;
            case LBM_P_VD_APLUS:
                if (!(v >= 0.0)) return fail(c, LBM_E_ARG, "van Driest A+ must be >= 0");
                c->vd_aplus = v;
                break;
            case LBM_P_VD_UTAU:
                if (!(v >= 0.0)) return fail(c, LBM_E_ARG, "van Driest friction velocity must be >= 0");
                c->vd_utau = v;
                break;
            case LBM_P_WALL_NODES:
                if (c->initialized)
                    return fail(c, LBM_E_STATE, "the wall placement is fixed once the state is initialised");
                if (v != 0.0 && v != 1.0 && v != 2.0)
                    return fail(c, LBM_E_ARG, "wall nodes is 0 (halfway walls), 1 or 2 (wall nodes, stress of the "
                                              "previous or of the same step)");
                if (c->wall_nodes != (int)v && c->dwn) {
                    drop_graphs(c);
                    (void)hipFree(c->dwn);
                    (void)hipFree(c->dwn_rec);
                    c->dwn = nullptr;
                    c->dwn_rec = nullptr;
                }
                c->wall_nodes = (int)v;
                break;
            default:
                return fail(c, LBM_E_ARG, "unknown or read-only parameter key");
        }
        c->cs2_dirty = true;
        drop_graphs(c);
        return LBM_OK;
    });
}

int lbm_get_param(const lbm_ctx* c, int key, double* v)
{
    return guard(const_cast<lbm_ctx*>(c), [&]() -> int {
        if (!c || !v) return fail(nullptr, LBM_E_ARG, "null argument");
        switch (key) {
            case LBM_P_Y1: *v = c->y1; break;
            case LBM_P_NEWTON_TOL: *v = c->newton_tol; break;
            case LBM_P_NEWTON_MAXIT: *v = c->newton_maxit; break;
            case LBM_P_STATS_EVERY: *v = c->stats_every; break;
            case LBM_P_STORE: *v = c->store; break;
            case LBM_P_TILE_ODD: *v = c->tile_odd; break;
            case LBM_P_TILE_EVEN: *v = c->tile_even; break;
            case LBM_P_XCD_REMAP: *v = c->xcd_remap; break;
            case LBM_P_XCD_CHUNK: *v = c->xcd_chunk; break;
            case LBM_P_VECTOR: *v = vector_width(c); break;
            case LBM_P_BRICK: *v = brick_rows(c); break;
            case LBM_P_ODD_ROWS: *v = c->odd_rows; break;
            case LBM_P_SPREAD: *v = spread_log2(c); break;
            case LBM_P_ODD_BY_ROWS: *v = odd_by_rows(c, c->odd_rows) ? 1.0 : 0.0; break;
            case LBM_P_COLLISION: *v = c->coll; break;
            case LBM_P_MRT_S_E:
            case LBM_P_MRT_S_EPS:
            case LBM_P_MRT_S_Q:
            case LBM_P_MRT_S_PI:
            case LBM_P_MRT_S_M: *v = c->mrt_s[key - LBM_P_MRT_S_E]; break;
            case LBM_P_VD_APLUS: *v = c->vd_aplus; break;
            case LBM_P_VD_UTAU: *v = c->vd_utau; break;
            case LBM_P_WALL_NODES: *v = c->wall_nodes; break;
            case LBM_P_GRAPH_STEPS: *v = c->graph_steps; break;
            case LBM_P_BC: *v = c->bc; break;
            case LBM_P_TAU0: *v = c->tau0; break;
            case LBM_P_FX: *v = c->fx; break;
            case LBM_P_CS: *v = c->cs; break;
            default: return fail(const_cast<lbm_ctx*>(c), LBM_E_ARG, "unknown parameter key");
        }
        return LBM_OK;
    });
}

int lbm_required_bytes(const lbm_ctx* c, size_t* bytes)
{
    return guard(const_cast<lbm_ctx*>(c), [&]() -> int {
        if (!c || !bytes) return fail(nullptr, LBM_E_ARG, "null argument");
        *bytes = (size_t)19 * (size_t)c->n * (size_t)store_bytes(c->store);
        return LBM_OK;
    });
}

int lbm_bind_storage(lbm_ctx* c, void* ptr, size_t bytes)
{
    return guard(c, [&]() -> int {
        if (!c || !ptr) return fail(c, LBM_E_ARG, "null argument");
        size_t need = 0;
        lbm_required_bytes(c, &need);
        if (bytes < need) return fail(c, LBM_E_ARG, "storage too small: need " + std::to_string(need) + " bytes");
        if (((uintptr_t)ptr) % 256 != 0) return fail(c, LBM_E_ARG, "storage must be 256-byte aligned");
        const int dev = device_of(ptr);
        if (dev < 0) return fail(c, LBM_E_ARG, "storage is not device memory");
        if (c->h && dev != c->dev) return fail(c, LBM_E_STATE, "storage must stay on the same device");
        c->dev = dev;
        DeviceGuard dg(c->dev);
        {
            // set-up of the device's work area for lbm_wall_yplus_pdf_noalloc (a failed
            // look-up is kept and reported by that call)
            double* ws = nullptr;
            (void)scratch_address(c->dev, &ws);
        }
        if (!c->dflags) {
            LBM_HIP(c, hipMalloc((void**)&c->dflags, sizeof(DevFlags)));
            LBM_HIP(c, hipMalloc((void**)&c->dacc, (size_t)c->ny * 8 * sizeof(double)));
            LBM_HIP(c, hipMalloc((void**)&c->dprof, (size_t)c->ny * sizeof(double)));
            LBM_HIP(c, hipMalloc((void**)&c->dcs2, (size_t)c->ny * sizeof(double)));
            LBM_HIP(c, hipMemset(c->dacc, 0, (size_t)c->ny * 8 * sizeof(double)));
            c->cs2_dirty = true;
        }
        drop_graphs(c);
        c->h = ptr;
        c->bytes = bytes;
        c->initialized = false;
        return LBM_OK;
    });
}

int lbm_set_stream(lbm_ctx* c, void* s)
{
    return guard(c, [&]() -> int {
        if (!c) return fail(nullptr, LBM_E_ARG, "null context");
        c->stream = (hipStream_t)s;
        return LBM_OK;
    });
}

int lbm_set_boundary(lbm_ctx* c, int bc)
{
    return guard(c, [&]() -> int {
        if (!c) return fail(nullptr, LBM_E_ARG, "null context");
        if (c->batch_member) return fail(c, LBM_E_STATE, "a batch instance's boundary is fixed at batch creation");
        if (bc != LBM_BB && bc != LBM_WFB && bc != LBM_FREESLIP) return fail(c, LBM_E_ARG, "unknown boundary");
        DeviceGuard dg(c->dev);
        c->bc = bc;
        drop_graphs(c);
        return fix_layout(c);
    });
}

static int init_spalding_impl(lbm_ctx* c, double u_tau, double noise, uint64_t seed);

int lbm_init_spalding(lbm_ctx* c, double u_tau, double noise, uint64_t seed)
{
    return guard(c, [&]() -> int {
        if (!c) return fail(nullptr, LBM_E_ARG, "null context");
        if (c->batch_member) return fail(c, LBM_E_STATE, "a batch instance is initialised through its batch");
        return init_spalding_impl(c, u_tau, noise, seed);
    });
}

static int init_spalding_impl(lbm_ctx* c, double u_tau, double noise, uint64_t seed)
{
    if (!c->h) return fail(c, LBM_E_STATE, "no storage bound");
    if (!std::isfinite(u_tau) || u_tau < 0.0 || !std::isfinite(noise) || noise < 0.0 || noise >= 1.0)
        return fail(c, LBM_E_ARG, "need 0 <= u_tau, 0 <= noise < 1");
    DeviceGuard dg(c->dev);
    std::vector<double> prof(c->ny);
    const double nu0 = (c->tau0 - 0.5) / 3.0;
    for (int y = 0; y < c->ny; ++y) {
        const int d = std::min(y, c->ny - 1 - y);
        const double dist = d + c->y1;
        prof[y] = u_tau * spalding_uplus_host(dist * u_tau / nu0, c->kappa, c->bconst);
    }
    LBM_HIP(c, hipMemcpyAsync(c->dprof, prof.data(), prof.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    c->brick = brick_for_tiles(c);
    LBM_HIP(c, launch_init_spalding(c->store, c->h, c->n, c->nx, c->ny, c->nz, c->brick, c->dprof, noise,
                                    (unsigned long long)seed, c->stream));
    c->steps = 0;
    c->layout_s = 0;
    c->layout_spec = (c->bc != kBB);
    c->initialized = true;
    int st = reset_flags(c);
    if (st == LBM_OK) st = start_wall_nodes(c);
    if (st != LBM_OK) return st;
    LBM_HIP(c, hipStreamSynchronize(c->stream));  // the profile lives on the host stack
    return LBM_OK;
}

int lbm_init_moments(lbm_ctx* c, const double* rho, const double* u)
{
    return guard(c, [&]() -> int {
        if (!c || !rho || !u) return fail(c, LBM_E_ARG, "null argument");
        if (c->batch_member) return fail(c, LBM_E_STATE, "a batch instance is initialised through its batch");
        if (!c->h) return fail(c, LBM_E_STATE, "no storage bound");
        for (long long i = 0; i < c->n; ++i) {
            const double r = rho[i], x = u[i], y = u[c->n + i], z = u[2 * c->n + i];
            if (!(r > 0.0) || !std::isfinite(r) || !std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z))
                return fail(c, LBM_E_ARG, "need finite moments and rho > 0");
        }
        DeviceGuard dg(c->dev);
        const long long chunk = std::min<long long>(c->n, 1ll << 24);
        std::vector<double> stage((size_t)chunk * 4);   // host staging first: a throw leaks no device memory
        double* tmp = nullptr;
        LBM_HIP(c, hipMalloc((void**)&tmp, (size_t)chunk * 4 * sizeof(double)));
        c->initialized = false;  // the layout is chosen afresh
        c->brick = brick_for_tiles(c);
        int st = LBM_OK;
        for (long long first = 0; first < c->n && st == LBM_OK; first += chunk) {
            const long long cnt = std::min(chunk, c->n - first);
            std::memcpy(stage.data(), rho + first, (size_t)cnt * sizeof(double));
            for (int k = 0; k < 3; ++k)
                std::memcpy(stage.data() + (size_t)(k + 1) * cnt, u + (size_t)k * c->n + first, (size_t)cnt * sizeof(double));
            hipError_t e = hipMemcpyAsync(tmp, stage.data(), (size_t)cnt * 4 * sizeof(double), hipMemcpyHostToDevice,
                                          c->stream);
            if (e == hipSuccess)
                e = launch_init_moments(c->store, c->h, c->n, c->nx, c->ny, c->nz, c->brick, first, cnt, tmp, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) st = fail(c, LBM_E_DEVICE, std::string("init_moments: ") + hipGetErrorString(e));
        }
        (void)hipFree(tmp);
        if (st != LBM_OK) return st;
        c->steps = 0;
        c->layout_s = 0;
        c->layout_spec = (c->bc != kBB);
        c->initialized = true;
        st = reset_flags(c);
        if (st == LBM_OK) st = start_wall_nodes(c);
        if (st != LBM_OK) return st;
        LBM_HIP(c, hipStreamSynchronize(c->stream));
        return LBM_OK;
    });
}

int lbm_set_state(lbm_ctx* c, const double* in, int64_t steps)
{
    return guard(c, [&]() -> int {
        if (!c || !in) return fail(c, LBM_E_ARG, "null argument");
        if (c->batch_member) return fail(c, LBM_E_STATE, "a batch instance's state is set through its batch");
        if (!c->h) return fail(c, LBM_E_STATE, "no storage bound");
        if (steps < 0) return fail(c, LBM_E_ARG, "steps must be >= 0");
        DeviceGuard dg(c->dev);
        const long long chunk = std::min<long long>(c->n, 1ll << 24);
        std::vector<double> stage((size_t)chunk * 19);  // host staging first: a throw leaks no device memory
        double* tmp = nullptr;
        LBM_HIP(c, hipMalloc((void**)&tmp, (size_t)chunk * 19 * sizeof(double)));
        c->initialized = false;  // the layout is chosen afresh
        c->brick = brick_for_tiles(c);
        int st = LBM_OK;
        for (long long first = 0; first < c->n && st == LBM_OK; first += chunk) {
            const long long cnt = std::min(chunk, c->n - first);
            for (int a = 0; a < 19; ++a)
                std::memcpy(stage.data() + (size_t)a * cnt, in + (size_t)a * c->n + first, (size_t)cnt * sizeof(double));
            hipError_t e = hipMemcpyAsync(tmp, stage.data(), (size_t)cnt * 19 * sizeof(double), hipMemcpyHostToDevice,
                                          c->stream);
            if (e == hipSuccess)
                e = launch_set_state(c->store, c->h, c->n, c->nx, c->ny, c->nz, c->brick, first, cnt, tmp, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) st = fail(c, LBM_E_DEVICE, std::string("set_state: ") + hipGetErrorString(e));
        }
        (void)hipFree(tmp);
        if (st != LBM_OK) return st;
        c->steps = steps;
        c->layout_s = 0;
        c->layout_spec = (c->bc != kBB);
        c->initialized = true;
        st = reset_flags(c);
        if (st == LBM_OK) st = start_wall_nodes(c);
        if (st != LBM_OK) return st;
        LBM_HIP(c, hipStreamSynchronize(c->stream));
        return LBM_OK;
    });
}

static int get_state_impl(lbm_ctx* c, long long count, const int64_t* cells, double* out)
{
    int st = check_ready(c);
    if (st != LBM_OK) return st;
    DeviceGuard dg(c->dev);
    if ((st = fix_layout(c)) != LBM_OK) return st;
    if ((st = sync_check(c)) != LBM_OK) return st;
    if (cells)
        for (long long i = 0; i < count; ++i)
            if (cells[i] < 0 || cells[i] >= c->n) return fail(c, LBM_E_ARG, "cell index out of range");
    const long long chunk = std::min<long long>(std::max<long long>(count, 1), 1ll << 24);
    std::vector<double> stage((size_t)chunk * 19);  // host buffers first: a throw leaks no device memory
    std::vector<double> result((size_t)count * 19);
    double* tmp = nullptr;
    long long* dcells = nullptr;
    LBM_HIP(c, hipMalloc((void**)&tmp, (size_t)chunk * 19 * sizeof(double)));
    if (cells && hipMalloc((void**)&dcells, (size_t)chunk * sizeof(long long)) != hipSuccess) {
        (void)hipFree(tmp);
        return fail(c, LBM_E_DEVICE, "get_state: allocation failed");
    }
    for (long long first = 0; first < count && st == LBM_OK; first += chunk) {
        const long long cnt = std::min(chunk, count - first);
        hipError_t e = hipSuccess;
        if (cells)
            e = hipMemcpyAsync(dcells, cells + first, (size_t)cnt * sizeof(long long), hipMemcpyHostToDevice,
                               c->stream);
        if (e == hipSuccess)
            e = launch_get_state(c->store, c->h, c->n, c->nx, c->ny, c->nz, c->brick, c->layout_s, c->layout_spec,
                                 cells ? dcells : nullptr, cells ? 0 : first, cnt, tmp, c->wall_nodes ? c->dwn : nullptr,
                                 c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(stage.data(), tmp, (size_t)cnt * 19 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            st = fail(c, LBM_E_DEVICE, std::string("get_state: ") + hipGetErrorString(e));
            break;
        }
        for (int a = 0; a < 19; ++a)
            std::memcpy(result.data() + (size_t)a * count + first, stage.data() + (size_t)a * cnt,
                        (size_t)cnt * sizeof(double));
    }
    (void)hipFree(tmp);
    if (dcells) (void)hipFree(dcells);
    if (st == LBM_OK) std::memcpy(out, result.data(), result.size() * sizeof(double));
    return st;
}

int lbm_get_state(lbm_ctx* c, double* out)
{
    return guard(c, [&]() -> int {
        if (!c || !out) return fail(c, LBM_E_ARG, "null argument");
        return get_state_impl(c, c->n, nullptr, out);
    });
}

int lbm_get_state_cells(lbm_ctx* c, int64_t n, const int64_t* cells, double* out)
{
    return guard(c, [&]() -> int {
        if (!c || !cells || !out || n < 0) return fail(c, LBM_E_ARG, "bad argument");
        if (n == 0) return LBM_OK;
        return get_state_impl(c, n, cells, out);
    });
}

// The per-row Smagorinsky factor 18 Cs^2 (1 - exp(-y+/A+))^2 with
// y+ = d u_tau / nu0, d = min(y, ny - 1 - y) + y1 (the first-layer distance
// rule) and u_tau the given friction velocity or sqrt(|Fx| ny / 2) from the
// force balance; uploaded in stream order when a parameter changed.
static int refresh_damping(lbm_ctx* c, hipStream_t s)
{
    if (!(c->vd_aplus > 0.0) || !c->cs2_dirty) return LBM_OK;
    const double nu0 = (c->tau0 - 0.5) / 3.0;
    const double ut = c->vd_utau > 0.0 ? c->vd_utau : std::sqrt(std::fabs(c->fx) * c->ny / 2.0);
    LBM_HIP(c, hipStreamSynchronize(s));   // no step still reads the old table
    c->hcs2.resize((size_t)c->ny);
    for (int y = 0; y < c->ny; ++y) {
        const int dy = std::min(y, c->ny - 1 - y);
        const double d = (double)dy + c->y1;
        const double ce = c->cs * (1.0 - std::exp(-(d * ut / nu0) / c->vd_aplus));
        c->hcs2[(size_t)y] = 18.0 * ce * ce;
    }
    LBM_HIP(c, hipMemcpyAsync(c->dcs2, c->hcs2.data(), (size_t)c->ny * sizeof(double), hipMemcpyHostToDevice, s));
    c->cs2_dirty = false;
    return LBM_OK;
}

int lbm_step(lbm_ctx* c, int64_t n)
{
    return guard(c, [&]() -> int {
        int st = check_ready(c);
        if (st != LBM_OK) return st;
        if (c->batch_member) return fail(c, LBM_E_STATE, "a batch instance is stepped by lbm_batch_step");
        if (n < 0) return fail(c, LBM_E_ARG, "n must be >= 0");
        if (n == 0) return LBM_OK;
        DeviceGuard dg(c->dev);
        if ((st = fix_layout(c)) != LBM_OK) return st;
        if ((st = ensure_partials(c)) != LBM_OK) return st;
        if ((st = refresh_damping(c, c->stream)) != LBM_OK) return st;
        long long left = n;
        while (left > 0) {
            if (c->graph_steps > 0 && left >= c->graph_steps) {
                const long long L = c->graph_steps;
                GraphKey key{c->layout_s, (int)L, c->stats_every, c->stats_every > 0 ? c->steps % c->stats_every : 0};
                auto it = c->graphs.find(key);
                if (it == c->graphs.end()) {
                    if (!c->cap_stream) LBM_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
                    hipGraph_t g = nullptr;
                    LBM_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
                    hipError_t e = enqueue_steps(c, c->cap_stream, c->layout_s, c->steps, L);
                    hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
                    if (e != hipSuccess || e2 != hipSuccess) {
                        if (g) (void)hipGraphDestroy(g);
                        return fail(c, LBM_E_DEVICE, std::string("graph capture: ") +
                                                         hipGetErrorString(e != hipSuccess ? e : e2));
                    }
                    hipGraphExec_t ex = nullptr;
                    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(g);
                    if (e != hipSuccess) return fail(c, LBM_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
                    try {
                        it = c->graphs.emplace(key, ex).first;
                    } catch (...) {
                        (void)hipGraphExecDestroy(ex);
                        throw;
                    }
                }
                LBM_HIP(c, hipGraphLaunch(it->second, c->stream));
                advance_bookkeeping(c, L);
                left -= L;
            } else {
                LBM_HIP(c, enqueue_steps(c, c->stream, c->layout_s, c->steps, 1));
                advance_bookkeeping(c, 1);
                left -= 1;
            }
        }
        return LBM_OK;
    });
}

int lbm_sync(lbm_ctx* c, int64_t* first_bad)
{
    return guard(c, [&]() -> int {
        if (!c) return fail(nullptr, LBM_E_ARG, "null context");
        if (first_bad) *first_bad = -1;
        if (!c->dflags) return LBM_OK;
        DeviceGuard dg(c->dev);
        DevFlags f;
        int st = read_flags(c, &f);
        if (st != LBM_OK) return st;
        st = status_of(f);
        if (st != LBM_OK) {
            if (first_bad) *first_bad = (int64_t)f.first_bad;
            return fail(c, st, std::string(lbm_status_str(st)) + " at step " + std::to_string((long long)f.first_bad));
        }
        return LBM_OK;
    });
}

int lbm_steps_done(const lbm_ctx* c, int64_t* s)
{
    return guard(const_cast<lbm_ctx*>(c), [&]() -> int {
        if (!c || !s) return fail(nullptr, LBM_E_ARG, "null argument");
        *s = c->steps;
        return LBM_OK;
    });
}

static int observe_impl(lbm_ctx* c, int mode, long long count, const int64_t* cells, double* out, int* iters,
                        double* dmass = nullptr)
{
    int st = check_ready(c);
    if (st != LBM_OK) return st;
    DeviceGuard dg(c->dev);
    if ((st = fix_layout(c)) != LBM_OK) return st;
    if ((st = sync_check(c)) != LBM_OK) return st;
    if (cells)
        for (long long i = 0; i < count; ++i)
            if (cells[i] < 0 || cells[i] >= c->n) return fail(c, LBM_E_ARG, "cell index out of range");
    const long long chunk = std::min<long long>(std::max<long long>(count, 1), 1ll << 24);
    std::vector<double> result((size_t)count * 4);  // host buffers first: a throw leaks no device memory
    std::vector<int> itres(iters ? (size_t)count : 0);
    std::vector<double> dmres(dmass ? (size_t)count * 2 : 0);
    double* tmp = nullptr;
    long long* dcells = nullptr;
    int* dit = nullptr;
    LBM_HIP(c, hipMalloc((void**)&tmp, (size_t)chunk * 4 * sizeof(double)));
    hipError_t e = hipSuccess;
    if (cells) e = hipMalloc((void**)&dcells, (size_t)chunk * sizeof(long long));
    if (e == hipSuccess && iters) e = hipMalloc((void**)&dit, (size_t)chunk * sizeof(int));
    double* ddm = nullptr;
    if (e == hipSuccess && dmass) e = hipMalloc((void**)&ddm, (size_t)chunk * 2 * sizeof(double));
    for (long long first = 0; first < count && e == hipSuccess; first += chunk) {
        const long long cnt = std::min(chunk, count - first);
        ObsArgs a = obs_args(c);
        a.mode = mode;
        a.cells = cells ? dcells : nullptr;
        a.first = cells ? 0 : first;
        a.count = cnt;
        a.out = tmp;
        a.iters = dit;
        a.dmass = ddm;
        if (cells)
            e = hipMemcpyAsync(dcells, cells + first, (size_t)cnt * sizeof(long long), hipMemcpyHostToDevice,
                               c->stream);
        if (mode == 1 && first != 0) e = hipErrorInvalidValue;  // wall records come in one chunk
        if (e == hipSuccess) e = launch_observe(c->store, a, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(result.data() + (size_t)first * 4, tmp, (size_t)cnt * 4 * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess && iters)
            e = hipMemcpyAsync(itres.data() + first, dit, (size_t)cnt * sizeof(int), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess && dmass)
            e = hipMemcpyAsync(dmres.data() + (size_t)first * 2, ddm, (size_t)cnt * 2 * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    (void)hipFree(tmp);
    if (dcells) (void)hipFree(dcells);
    if (dit) (void)hipFree(dit);
    if (ddm) (void)hipFree(ddm);
    if (e != hipSuccess) return fail(c, LBM_E_DEVICE, std::string("observe: ") + hipGetErrorString(e));
    std::memcpy(out, result.data(), result.size() * sizeof(double));
    if (iters) std::memcpy(iters, itres.data(), itres.size() * sizeof(int));
    if (dmass) std::memcpy(dmass, dmres.data(), dmres.size() * sizeof(double));
    return LBM_OK;
}

int lbm_moments(lbm_ctx* c, double* rho, double* ux, double* uy, double* uz)
{
    return guard(c, [&]() -> int {
        if (!c) return fail(nullptr, LBM_E_ARG, "null context");
        std::vector<double> buf;
        try {
            buf.resize((size_t)c->n * 4);
        } catch (...) {
            return fail(c, LBM_E_OOM, "host buffer allocation failed");
        }
        int st = observe_impl(c, 0, c->n, nullptr, buf.data(), nullptr);
        if (st != LBM_OK) return st;
        for (long long i = 0; i < c->n; ++i) {
            if (rho) rho[i] = buf[4 * i];
            if (ux) ux[i] = buf[4 * i + 1];
            if (uy) uy[i] = buf[4 * i + 2];
            if (uz) uz[i] = buf[4 * i + 3];
        }
        return LBM_OK;
    });
}

int lbm_moments_device(lbm_ctx* c, double* rho, double* ux, double* uy, double* uz)
{
    return guard(c, [&]() -> int {
        int st = check_ready(c);
        if (st != LBM_OK) return st;
        double* outs[4] = {rho, ux, uy, uz};
        bool any = false;
        for (double* p : outs) {
            if (!p) continue;
            any = true;
            if (device_of(p) != c->dev)
                return fail(c, LBM_E_ARG, "moment arrays must be device memory on the context's device");
        }
        if (!any) return fail(c, LBM_E_ARG, "no output array given");
        DeviceGuard dg(c->dev);
        if ((st = fix_layout(c)) != LBM_OK) return st;
        ObsArgs a = obs_args(c);
        a.mode = 0;
        a.cells = nullptr;
        a.first = 0;
        a.count = c->n;
        a.out = nullptr;
        for (int k = 0; k < 4; ++k) a.soa[k] = outs[k];
        a.iters = nullptr;
        a.dmass = nullptr;
        LBM_HIP(c, launch_observe(c->store, a, c->stream));
        return LBM_OK;
    });
}

int lbm_moments_cells(lbm_ctx* c, int64_t n, const int64_t* cells, double* out)
{
    return guard(c, [&]() -> int {
        if (!c || !cells || !out || n < 0) return fail(c, LBM_E_ARG, "bad argument");
        if (n == 0) return LBM_OK;
        return observe_impl(c, 0, n, cells, out, nullptr);
    });
}

int lbm_wall_shear(lbm_ctx* c, double* tx, double* tz, double* ut, double* U)
{
    return guard(c, [&]() -> int {
        if (!c) return fail(nullptr, LBM_E_ARG, "null context");
        const long long m = 2ll * c->nx * c->nz;
        std::vector<double> buf((size_t)m * 4);
        int st = observe_impl(c, 1, m, nullptr, buf.data(), nullptr);
        if (st != LBM_OK) return st;
        for (long long i = 0; i < m; ++i) {
            if (tx) tx[i] = buf[4 * i];
            if (tz) tz[i] = buf[4 * i + 1];
            if (ut) ut[i] = buf[4 * i + 2];
            if (U) U[i] = buf[4 * i + 3];
        }
        return LBM_OK;
    });
}

int lbm_wall_mass_change(lbm_ctx* c, double* dsum, double* rho)
{
    return guard(c, [&]() -> int {
        if (!c) return fail(nullptr, LBM_E_ARG, "null context");
        if (!dsum && !rho) return fail(c, LBM_E_ARG, "null argument");
        if (c->wall_nodes) return fail(c, LBM_E_STATE, "the mass check is defined for the first-layer correction of halfway walls");
        const long long m = 2ll * c->nx * c->nz;
        std::vector<double> buf((size_t)m * 4), dm((size_t)m * 2);
        int st = observe_impl(c, 1, m, nullptr, buf.data(), nullptr, dm.data());
        if (st != LBM_OK) return st;
        for (long long i = 0; i < m; ++i) {
            if (dsum) dsum[i] = dm[2 * i];
            if (rho) rho[i] = dm[2 * i + 1];
        }
        return LBM_OK;
    });
}

// The y+ distribution's kernels on the context's stream: the wall records'
// friction velocities into ut[2 nx nz], then the moments into ms[2] and the
// histogram into counts[nbins + 2] (cleared by the kernels).
static hipError_t enqueue_yplus_pdf(lbm_ctx* c, int nbins, double lo, double hi, double* ut, double* ms,
                                    unsigned long long* counts)
{
    const long long m = 2ll * c->nx * c->nz;
    ObsArgs a = obs_args(c);
    a.mode = 1;
    a.cells = nullptr;
    a.first = 0;
    a.count = m;
    a.out = nullptr;
    a.soa[2] = ut;
    a.iters = nullptr;
    a.dmass = nullptr;
    hipError_t e = launch_observe(c->store, a, c->stream);
    if (e != hipSuccess) return e;
    const double nu0 = (c->tau0 - 0.5) / 3.0;
    return launch_yplus_pdf(ut, m, c->y1, nu0, ms, lo, (double)nbins / (hi - lo), nbins, counts, c->stream);
}

int lbm_wall_yplus_pdf(lbm_ctx* c, int32_t nbins, double lo, double hi, int64_t* counts, double* mean_std)
{
    return guard(c, [&]() -> int {
        if (!c || !counts || !mean_std) return fail(c, LBM_E_ARG, "null argument");
        if (nbins < 1 || nbins > (1 << 20) || !(hi > lo) || !std::isfinite(lo) || !std::isfinite(hi))
            return fail(c, LBM_E_ARG, "need 1 <= nbins <= 2^20 and finite lo < hi");
        int st = check_ready(c);
        if (st != LBM_OK) return st;
        DeviceGuard dg(c->dev);
        if ((st = fix_layout(c)) != LBM_OK) return st;
        if ((st = sync_check(c)) != LBM_OK) return st;
        const long long m = 2ll * c->nx * c->nz;
        std::vector<unsigned long long> hc((size_t)nbins + 2);  // host buffer first: a throw leaks no device memory
        double* ut = nullptr;
        double* ms = nullptr;
        unsigned long long* dcnt = nullptr;
        hipError_t e = hipMalloc((void**)&ut, (size_t)m * sizeof(double));
        if (e == hipSuccess) e = hipMalloc((void**)&ms, 2 * sizeof(double));
        if (e == hipSuccess) e = hipMalloc((void**)&dcnt, (size_t)(nbins + 2) * sizeof(unsigned long long));
        double hms[2] = {0.0, 0.0};
        if (e == hipSuccess) e = enqueue_yplus_pdf(c, nbins, lo, hi, ut, ms, dcnt);
        if (e == hipSuccess) e = hipMemcpyAsync(hms, ms, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hc.data(), dcnt, hc.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (ut) (void)hipFree(ut);
        if (ms) (void)hipFree(ms);
        if (dcnt) (void)hipFree(dcnt);
        if (e != hipSuccess) return fail(c, LBM_E_DEVICE, std::string("wall y+ distribution: ") + hipGetErrorString(e));
        for (size_t i = 0; i < hc.size(); ++i) counts[i] = (int64_t)hc[i];
        mean_std[0] = hms[0];
        mean_std[1] = hms[1];
        return LBM_OK;
    });
}

int lbm_wall_yplus_pdf_noalloc(lbm_ctx* c, int32_t nbins, double lo, double hi, int64_t* counts, double* mean_std)
{
    return guard(c, [&]() -> int {
        if (!c || !counts || !mean_std) return fail(c, LBM_E_ARG, "null argument");
        if (nbins < 1 || nbins > (1 << 20) || !(hi > lo) || !std::isfinite(lo) || !std::isfinite(hi))
            return fail(c, LBM_E_ARG, "need 1 <= nbins <= 2^20 and finite lo < hi");
        const long long m = 2ll * c->nx * c->nz;
        if (m > kScratchWallCells)
            return fail(c, LBM_E_ARG, "2 nx nz = " + std::to_string(m) + " wall cells exceed the fixed work area of " +
                                          std::to_string(kScratchWallCells) + "; use lbm_wall_yplus_pdf");
        int st = check_ready(c);
        if (st != LBM_OK) return st;
        if (layout_stale(c))
            return fail(c, LBM_E_STATE, "the boundary changed since the last step and the state must be re-laid "
                                        "out first (lbm_step or lbm_wall_yplus_pdf does it)");
        const void* outs[2] = {counts, mean_std};
        for (const void* p : outs) {
            if (device_of(p) != c->dev)
                return fail(c, LBM_E_ARG, "counts and mean_std must be device memory on the context's device");
        }
        DeviceGuard dg(c->dev);
        double* ws = nullptr;
        const hipError_t e = scratch_address(c->dev, &ws);
        if (e != hipSuccess) return fail(c, LBM_E_DEVICE, std::string("work area look-up: ") + hipGetErrorString(e));
        LBM_HIP(c, enqueue_yplus_pdf(c, nbins, lo, hi, ws, mean_std, (unsigned long long*)counts));
        return LBM_OK;
    });
}

int lbm_get_wall_nodes(lbm_ctx* c, double* fw, double* rec)
{
    return guard(c, [&]() -> int {
        int st = check_ready(c);
        if (st != LBM_OK) return st;
        if (!c->wall_nodes) return fail(c, LBM_E_STATE, "the context has no wall nodes");
        if (!fw && !rec) return fail(c, LBM_E_ARG, "null argument");
        DeviceGuard dg(c->dev);
        if ((st = sync_check(c)) != LBM_OK) return st;
        const size_t m = (size_t)2 * c->nx * c->nz;
        std::vector<double> hf(fw ? 5 * m : 0), hr(rec ? 4 * m : 0);
        double* tmp = nullptr;
        hipError_t e = hipSuccess;
        if (fw) {
            e = hipMalloc((void**)&tmp, 5 * m * sizeof(double));
            if (e == hipSuccess) e = launch_node_get(c->store, c->dwn, c->layout_s, c->nx, c->nz, tmp, c->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(hf.data(), tmp, 5 * m * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        }
        if (e == hipSuccess && rec)
            e = hipMemcpyAsync(hr.data(), c->dwn_rec, 4 * m * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (tmp) (void)hipFree(tmp);
        if (e != hipSuccess) return fail(c, LBM_E_DEVICE, std::string("wall nodes: ") + hipGetErrorString(e));
        if (fw) std::memcpy(fw, hf.data(), hf.size() * sizeof(double));
        if (rec) std::memcpy(rec, hr.data(), hr.size() * sizeof(double));
        return LBM_OK;
    });
}

int lbm_stats_reset(lbm_ctx* c)
{
    return guard(c, [&]() -> int {
        if (!c) return fail(nullptr, LBM_E_ARG, "null context");
        if (!c->dacc) return fail(c, LBM_E_STATE, "no storage bound");
        DeviceGuard dg(c->dev);
        LBM_HIP(c, hipStreamSynchronize(c->stream));
        LBM_HIP(c, hipMemset(c->dacc, 0, (size_t)c->ny * 8 * sizeof(double)));
        c->nsamples = 0;
        return LBM_OK;
    });
}

int lbm_stats_sums(lbm_ctx* c, double* out, int64_t* nsamples)
{
    return guard(c, [&]() -> int {
        if (!c || !out) return fail(c, LBM_E_ARG, "null argument");
        if (!c->dacc) return fail(c, LBM_E_STATE, "no storage bound");
        DeviceGuard dg(c->dev);
        int st = sync_check(c);
        if (st != LBM_OK) return st;
        LBM_HIP(c, hipMemcpy(out, c->dacc, (size_t)c->ny * 8 * sizeof(double), hipMemcpyDeviceToHost));
        if (nsamples) *nsamples = c->nsamples;
        return LBM_OK;
    });
}

int lbm_stats_get(lbm_ctx* c, double* out, int64_t* nsamples)
{
    return guard(c, [&]() -> int {
        if (!c || !out) return fail(c, LBM_E_ARG, "null argument");
        std::vector<double> s((size_t)c->ny * 8);
        int st = lbm_stats_sums(c, s.data(), nsamples);
        if (st != LBM_OK) return st;
        for (int y = 0; y < c->ny; ++y) {
            const double* r = &s[(size_t)y * 8];
            double* o = out + (size_t)y * 8;
            const double m = r[7];
            if (m <= 0.0) {
                for (int k = 0; k < 8; ++k) o[k] = 0.0;
                continue;
            }
            const double mx = r[0] / m, my = r[1] / m, mz = r[2] / m;
            o[0] = mx; o[1] = my; o[2] = mz;
            o[3] = r[3] / m - mx * mx;
            o[4] = r[4] / m - my * my;
            o[5] = r[5] / m - mz * mz;
            o[6] = r[6] / m - mx * my;
            o[7] = m;
        }
        return LBM_OK;
    });
}

namespace {

// Launch shapes of a single channel: block sizes of the odd and even kernels,
// cells per thread, rows per brick requested (0 = automatic), launch order
// (LBM_P_SPREAD), the odd-step mode (LBM_P_ODD_ROWS) and the XCD chunk
// (LBM_P_XCD_CHUNK).
struct Shapes {
    int tile_odd, tile_even, vw, brick, spread, odd_rows, xcd;
    bool operator==(const Shapes& o) const
    {
        return std::tie(tile_odd, tile_even, vw, brick, spread, odd_rows, xcd) ==
               std::tie(o.tile_odd, o.tile_even, o.vw, o.brick, o.spread, o.odd_rows, o.xcd);
    }
};

// The tuner's results, kept for the life of the process per device, grid,
// store, boundary, collision and wall placement.
struct TuneKey {
    int dev, nx, ny, nz, store, bc, coll, wall_nodes;
    bool operator<(const TuneKey& o) const
    {
        return std::tie(dev, nx, ny, nz, store, bc, coll, wall_nodes) <
               std::tie(o.dev, o.nx, o.ny, o.nz, o.store, o.bc, o.coll, o.wall_nodes);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, Shapes> g_tune_cache;

Shapes shapes_of(const lbm_ctx* c)
{
    return Shapes{c->tile_odd, c->tile_even, vector_width(c), c->brick_req, spread_log2(c), c->odd_rows, c->xcd_chunk};
}

void apply_shapes(lbm_ctx* c, const Shapes& v)
{
    c->tile_odd = v.tile_odd;
    c->tile_even = v.tile_even;
    c->vw_req = v.vw;
    c->brick_req = v.brick;
    c->spread = v.spread;
    c->odd_rows = v.odd_rows;
    c->xcd_chunk = v.xcd;
}

// What the odd and even launches of shapes v look like (geometry, order and
// kernel variant); two shapes with the same signature run the same kernels.
std::vector<long long> launch_signature(lbm_ctx* c, const Shapes& v)
{
    const Shapes keep = shapes_of(c);
    apply_shapes(c, v);
    std::vector<long long> sig;
    for (bool odd : {true, false}) {
        const StepArgs a = step_args(c, odd, c->odd_rows);
        for (long long x : {(long long)a.brick, (long long)a.spread, (long long)a.spread_rot, (long long)a.nseg,
                            (long long)a.tile_x, (long long)a.vw, (long long)a.ntx, (long long)a.rpb,
                            (long long)a.nyt, (long long)a.ntiles, (long long)a.xcd_remap})
            sig.push_back(x);
    }
    apply_shapes(c, keep);
    return sig;
}

bool same_launch(lbm_ctx* c, const Shapes& a, const Shapes& b)
{
    return launch_signature(c, a) == launch_signature(c, b);
}

}  // namespace

int lbm_autotune(lbm_ctx* c, int steps, int32_t* out)
{
    return guard(c, [&]() -> int {
        if (!c) return fail(nullptr, LBM_E_ARG, "null context");
        if (c->batch_member) return fail(c, LBM_E_STATE, "a batch is tuned with lbm_batch_autotune");
        if (!c->h) return fail(c, LBM_E_STATE, "no storage bound");
        if (c->initialized) return fail(c, LBM_E_STATE, "autotune runs before the state is initialised");
        if (steps < 2) return fail(c, LBM_E_ARG, "steps must be >= 2");
        DeviceGuard dg(c->dev);
        const TuneKey key{c->dev, c->nx, c->ny, c->nz, c->store, c->bc, c->coll, c->wall_nodes};
        auto report = [&](const Shapes& v, bool cached) {
            if (out) {
                out[0] = v.tile_odd;
                out[1] = v.tile_even;
                out[2] = v.vw;
                out[3] = brick_for_tiles(c);
                out[4] = v.spread;
                out[5] = odd_by_rows(c, v.odd_rows) ? 1 : 0;
                out[6] = cached ? 1 : 0;
                out[7] = v.xcd;
            }
        };
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                apply_shapes(c, it->second);
                drop_graphs(c);
                report(it->second, true);
                return LBM_OK;
            }
        }
        // a representative state: the initial profile the body force implies,
        // written again whenever a candidate's rows per brick change the layout
        const double ut = std::sqrt(std::fabs(c->fx) * c->ny * 0.5);
        int state_brick = -1;
        TimingEvents tev;
        if (!tev.create()) return fail(c, LBM_E_DEVICE, "autotune: event creation failed");
        hipEvent_t* ev = tev.ev;
        const Shapes start = shapes_of(c);
        int st = LBM_OK;
        hipError_t err = hipSuccess;
        // mean odd and even kernel times (ms) of shapes v: one warm-up step pair,
        // then steps / 2 timed pairs
        auto measure = [&](const Shapes& v, float* to, float* te) -> bool {
            apply_shapes(c, v);
            if (brick_for_tiles(c) != state_brick) {
                if ((st = init_spalding_impl(c, ut, 0.05, 0)) != LBM_OK) return false;
                c->initialized = false;  // a timing state only: each candidate takes the layout its shapes want
                state_brick = c->brick;
            }
            const int pairs = std::max(1, steps / 2);
            *to = *te = 0.f;
            for (int r = 0; r <= pairs && err == hipSuccess; ++r) {
                const StepArgs ao = step_args(c, true, c->odd_rows), ae = step_args(c, false, c->odd_rows);
                err = hipEventRecord(ev[0], c->stream);
                if (err == hipSuccess) err = launch_step(c->store, true, c->bc, ao, c->stream);
                if (err == hipSuccess) err = hipEventRecord(ev[1], c->stream);
                if (err == hipSuccess) err = launch_step(c->store, false, c->bc, ae, c->stream);
                if (err == hipSuccess) err = hipEventRecord(ev[2], c->stream);
                if (err == hipSuccess) err = hipEventSynchronize(ev[2]);
                float a = 0.f, b = 0.f;
                if (err == hipSuccess) err = hipEventElapsedTime(&a, ev[0], ev[1]);
                if (err == hipSuccess) err = hipEventElapsedTime(&b, ev[1], ev[2]);
                if (r > 0) {
                    *to += a / pairs;
                    *te += b / pairs;
                }
            }
            return err == hipSuccess;
        };
        // Coordinate descent from the current shapes: one setting at a time, a
        // change kept only when it is faster by more than kMargin (timing noise);
        // the odd-step settings are decided by the odd kernel's time, the even block
        // size by the even kernel's, the shared settings by the pair's.
        constexpr float kMargin = 0.01f;
        Shapes best = start;
        float bo = 0.f, be = 0.f;
        bool ok = measure(best, &bo, &be);
        const int tiles[4] = {64, 128, 256, 512};
        const int widths[3] = {1, 2, 4};
        const int bricks[4] = {4, 8, 16, 32};
        const int spreads[4] = {0, 5, 7, 9};
        const int xcd_chunks[3] = {5, 7, 9};
        enum Criterion { kPair, kOdd, kEven };
        auto consider = [&](Shapes v, Criterion j) -> bool {
            if (!ok || same_launch(c, v, best)) return false;
            float to = 0.f, te = 0.f;
            if (!(ok = measure(v, &to, &te))) return false;
            const float was = j == kOdd ? bo : j == kEven ? be : bo + be;
            const float now = j == kOdd ? to : j == kEven ? te : to + te;
            if (now < was * (1.f - kMargin)) {
                best = v;
                if (j == kOdd) {
                    bo = to;
                } else if (j == kEven) {
                    be = te;
                } else {
                    bo = to;
                    be = te;
                }
                return true;
            }
            return false;
        };
        for (int round = 0; round < 2 && ok; ++round) {
            bool changed = false;
            for (int w : widths) {
                if (!step_vector_width_ok(c->store, c->nx, w)) continue;
                Shapes v = best;
                v.vw = w;
                changed |= consider(v, kPair);
            }
            for (int t : tiles) {
                Shapes v = best;
                v.tile_odd = t;
                changed |= consider(v, kOdd);
            }
            for (int m : {0, 2}) {
                Shapes v = best;
                v.odd_rows = m;
                changed |= consider(v, kOdd);
            }
            for (int t : tiles) {
                Shapes v = best;
                v.tile_even = t;
                changed |= consider(v, kEven);
            }
            for (int b : bricks) {
                Shapes v = best;
                v.brick = b;
                changed |= consider(v, kPair);
            }
            for (int sp : spreads) {
                Shapes v = best;
                v.spread = sp;
                changed |= consider(v, kPair);
            }
            for (int xc : xcd_chunks) {
                Shapes v = best;
                v.xcd = xc;
                changed |= consider(v, kPair);
            }
            if (!changed) break;
        }
        apply_shapes(c, ok ? best : start);
        c->initialized = false;
        drop_graphs(c);
        if (st != LBM_OK) return st;
        if (err != hipSuccess) return fail(c, LBM_E_DEVICE, std::string("autotune: ") + hipGetErrorString(err));
        DevFlags f;
        if ((st = read_flags(c, &f)) != LBM_OK) return st;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_cache[key] = best;
        }
        report(best, false);
        return LBM_OK;
    });
}

int lbm_spalding_uplus(double yplus, double kappa, double B, double* uplus)
{
    return guard(nullptr, [&]() -> int {
        if (!uplus || !std::isfinite(yplus) || yplus < 0.0 || !(kappa > 0.0) || !std::isfinite(B))
            return fail(nullptr, LBM_E_ARG, "need y+ >= 0, kappa > 0, finite B");
        *uplus = spalding_uplus_host(yplus, kappa, B);
        return LBM_OK;
    });
}

int lbm_device_wall_utau(int32_t n, const double* U, double y1, double nu, double kappa, double B, double tol,
                         int32_t maxit, double* ut, int32_t* iters)
{
    return guard(nullptr, [&]() -> int {
        if (n < 0 || (n > 0 && (!U || !ut || !iters))) return fail(nullptr, LBM_E_ARG, "bad argument");
        if (!(y1 > 0) || !(nu > 0) || !(kappa > 0) || !(tol > 0) || maxit < 1) return fail(nullptr, LBM_E_ARG, "bad parameter");
        if (n == 0) return LBM_OK;
        double *dU = nullptr, *dut = nullptr;
        int* dit = nullptr;
        hipError_t e = hipMalloc((void**)&dU, (size_t)n * sizeof(double));
        if (e == hipSuccess) e = hipMalloc((void**)&dut, (size_t)n * sizeof(double));
        if (e == hipSuccess) e = hipMalloc((void**)&dit, (size_t)n * sizeof(int));
        if (e == hipSuccess) e = hipMemcpy(dU, U, (size_t)n * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = launch_wall_utau(dU, n, y1, nu, kappa, B, tol, maxit, dut, dit, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e == hipSuccess) e = hipMemcpy(ut, dut, (size_t)n * sizeof(double), hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(iters, dit, (size_t)n * sizeof(int), hipMemcpyDeviceToHost);
        if (dU) (void)hipFree(dU);
        if (dut) (void)hipFree(dut);
        if (dit) (void)hipFree(dit);
        if (e != hipSuccess) return fail(nullptr, LBM_E_DEVICE, std::string("device wall solve: ") + hipGetErrorString(e));
        return LBM_OK;
    });
}

int lbm_codec_roundtrip(int store, int64_t n, const float* in, float* out)
{
    return guard(nullptr, [&]() -> int {
        if (store < 0 || store > 3 || n < 0 || (n > 0 && (!in || !out)))
            return fail(nullptr, LBM_E_ARG, "bad argument");
        if (n == 0) return LBM_OK;
        float *din = nullptr, *dout = nullptr;
        hipError_t e = hipMalloc((void**)&din, (size_t)n * sizeof(float));
        if (e == hipSuccess) e = hipMalloc((void**)&dout, (size_t)n * sizeof(float));
        if (e == hipSuccess) e = hipMemcpy(din, in, (size_t)n * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = launch_codec(store, din, dout, n, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e == hipSuccess) e = hipMemcpy(out, dout, (size_t)n * sizeof(float), hipMemcpyDeviceToHost);
        if (din) (void)hipFree(din);
        if (dout) (void)hipFree(dout);
        if (e != hipSuccess) return fail(nullptr, LBM_E_DEVICE, std::string("codec round trip: ") + hipGetErrorString(e));
        return LBM_OK;
    });
}

int lbm_copy_probe(void* dst, const void* src, size_t bytes, void* s)
{
    return guard(nullptr, [&]() -> int {
        if (!dst || !src || bytes % 16 != 0) return fail(nullptr, LBM_E_ARG, "need device pointers and bytes % 16 == 0");
        hipError_t e = launch_copy(src, dst, bytes, (hipStream_t)s);
        if (e != hipSuccess) return fail(nullptr, LBM_E_DEVICE, std::string("copy probe: ") + hipGetErrorString(e));
        return LBM_OK;
    });
}

}  // extern "C"

// ================================================================ batches

struct lbm_batch {
    int n = 0;
    std::vector<lbm_ctx*> inst;
    int store = kStoreF64;
    int tile_odd = 256, tile_even = 256, vw_req = 0, xcd_remap = 1, graph_steps = 32;
    int odd_rows = 1;            // as lbm_ctx::odd_rows, applied to every instance alike
    void* h = nullptr;
    size_t bytes = 0;
    int dev = -1;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    std::vector<size_t> offset;      // byte offset of each instance's populations
    std::vector<StepArgs> tab[2];    // [even, odd] per-instance launch parameters
    StepArgs* dtab[2] = {nullptr, nullptr};
    int* dmap[2] = {nullptr, nullptr};
    int ntiles[2] = {0, 0};
    bool tables_ready = false;
    bool initialized = false;
    long long steps = 0;
    int layout_s = 0;
    std::map<GraphKey, hipGraphExec_t> graphs;
    std::string err;
};

namespace {

int bfail(lbm_batch* b, int code, const std::string& msg)
{
    if (b) b->err = msg;
    else g_err = msg;
    return code;
}

int bfail_nothrow(lbm_batch* b, int code, const char* msg) noexcept
{
    try {
        if (b) b->err = msg;
        else g_err = msg;
    } catch (...) {
    }
    return code;
}

template <typename F>
int bguard(lbm_batch* b, F&& body) noexcept
{
    try {
        return body();
    } catch (const std::bad_alloc&) {
        return bfail_nothrow(b, LBM_E_OOM, "host memory allocation failed");
    } catch (...) {
        return bfail_nothrow(b, LBM_E_STATE, "internal error (exception)");
    }
}

#define LBM_BHIP(b, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return bfail((b), LBM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));  \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int batch_width(const lbm_batch* b)
{
    auto ok_all = [&](int vw) {
        for (const lbm_ctx* c : b->inst)
            if (!step_vector_width_ok(b->store, c->nx, vw)) return false;
        return true;
    };
    if (b->vw_req > 0 && ok_all(b->vw_req)) return b->vw_req;
    if (b->store == LBM_STORE_F32) return 1;   // as auto_vector_width
    for (int vw = 8 / store_bytes(b->store); vw > 1; vw /= 2)
        if (ok_all(vw)) return vw;
    return 1;
}

void batch_drop_graphs(lbm_batch* b)
{
    if (b->graphs.empty()) return;
    (void)hipStreamSynchronize(b->stream);
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
}

void batch_free_tables(lbm_batch* b)
{
    for (int k = 0; k < 2; ++k) {
        if (b->dtab[k]) (void)hipFree(b->dtab[k]);
        if (b->dmap[k]) (void)hipFree(b->dmap[k]);
        b->dtab[k] = nullptr;
        b->dmap[k] = nullptr;
        b->tab[k].clear();
        b->ntiles[k] = 0;
    }
    b->tables_ready = false;
}

// The batch's launch shapes on every instance.
void batch_apply_shapes(lbm_batch* b)
{
    const int vw = batch_width(b);
    for (lbm_ctx* c : b->inst) {
        c->vw_req = vw;
        c->tile_odd = b->tile_odd;
        c->tile_even = b->tile_even;
    }
}

// whether the batch's launch shapes fit the layouts of the instances' states
bool batch_shapes_fit(const lbm_batch* b)
{
    const int vw = batch_width(b);
    for (const lbm_ctx* c : b->inst) {
        if (!c->initialized) continue;
        if (!brick_ok(c->ny, c->brick, rows_per_block(c, b->tile_odd, vw)) ||
            !brick_ok(c->ny, c->brick, rows_per_block(c, b->tile_even, vw)))
            return false;
    }
    return true;
}

// Per-instance launch parameters and the tile -> instance map of both kernels.
int batch_tables(lbm_batch* b)
{
    if (b->tables_ready) return LBM_OK;
    batch_drop_graphs(b);
    batch_free_tables(b);
    batch_apply_shapes(b);
    // one odd kernel serves every instance: rows only if all of them qualify
    int rows_mode = b->odd_rows;
    for (const lbm_ctx* c : b->inst)
        if (!odd_by_rows(c, rows_mode)) rows_mode = 0;
    for (int k = 0; k < 2; ++k) {
        const bool odd = (k == 1);
        std::vector<int> map;
        int total = 0;
        for (int i = 0; i < b->n; ++i) {
            lbm_ctx* c = b->inst[i];
            StepArgs a = step_args(c, odd, rows_mode);
            a.tile_begin = total;
            total += a.ntiles;
            map.insert(map.end(), (size_t)a.ntiles, i);
            b->tab[k].push_back(a);
        }
        b->ntiles[k] = total;
        LBM_BHIP(b, hipMalloc((void**)&b->dtab[k], sizeof(StepArgs) * b->n));
        LBM_BHIP(b, hipMalloc((void**)&b->dmap[k], sizeof(int) * map.size()));
        LBM_BHIP(b, hipMemcpy(b->dtab[k], b->tab[k].data(), sizeof(StepArgs) * b->n, hipMemcpyHostToDevice));
        LBM_BHIP(b, hipMemcpy(b->dmap[k], map.data(), sizeof(int) * map.size(), hipMemcpyHostToDevice));
    }
    b->tables_ready = true;
    return LBM_OK;
}

hipError_t batch_enqueue(const lbm_batch* b, hipStream_t s, int layout_s, long long len)
{
    for (long long i = 0; i < len; ++i) {
        const int k = (layout_s == 0) ? 1 : 0;  // layout P -> odd kernel
        hipError_t e = launch_batch_step(b->store, k == 1, b->tab[k].data(), b->n, b->dtab[k], b->dmap[k],
                                         b->ntiles[k], b->xcd_remap ? kXcdChunkLog2 + 1 : 0, s);
        if (e != hipSuccess) return e;
        layout_s ^= 1;
    }
    return hipSuccess;
}

void batch_advance(lbm_batch* b, long long len)
{
    for (long long i = 0; i < len; ++i) {
        for (lbm_ctx* c : b->inst) {
            if (c->layout_s == 0) c->layout_spec = (c->bc != kBB);
            c->layout_s ^= 1;
            c->steps += 1;
        }
        b->layout_s ^= 1;
        b->steps += 1;
    }
}

}  // namespace

extern "C" {

int lbm_batch_create(int32_t n, const lbm_grid* grids, const double* tau, const double* Cs, const double* Fx,
                     const int32_t* bc, double kappa, double B, lbm_batch** out)
{
    return guard(nullptr, [&]() -> int {
        if (n < 1 || !grids || !tau || !Cs || !Fx || !bc || !out) return bfail(nullptr, LBM_E_ARG, "bad argument");
        for (int i = 0; i < n; ++i)
            if (bc[i] != LBM_BB && bc[i] != LBM_WFB && bc[i] != LBM_FREESLIP)
                return bfail(nullptr, LBM_E_ARG, "unknown boundary of instance " + std::to_string(i));
        lbm_batch* b = new (std::nothrow) lbm_batch();
        if (!b) return bfail(nullptr, LBM_E_OOM, "batch allocation failed");
        b->n = n;
        for (int i = 0; i < n; ++i) {
            lbm_ctx* c = nullptr;
            int st = lbm_create(&grids[i], tau[i], Cs[i], kappa, B, Fx[i], &c);
            if (st != LBM_OK) {
                std::string msg = "instance " + std::to_string(i) + ": " + g_err;
                for (lbm_ctx* q : b->inst) lbm_destroy(q);
                delete b;
                return bfail(nullptr, st, msg);
            }
            c->bc = bc[i];
            c->graph_steps = 0;
            b->inst.push_back(c);
        }
        *out = b;
        return LBM_OK;
    });
}

void lbm_batch_destroy(lbm_batch* b)
{
    if (!b) return;
    DeviceGuard dg(b->dev);
    if (b->h) (void)hipStreamSynchronize(b->stream);
    batch_drop_graphs(b);
    batch_free_tables(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (lbm_ctx* c : b->inst) lbm_destroy(c);
    delete b;
}

int lbm_batch_set_param(lbm_batch* b, int key, double v)
{
    return bguard(b, [&]() -> int {
        if (!b) return bfail(nullptr, LBM_E_ARG, "null batch");
        if (!std::isfinite(v)) return bfail(b, LBM_E_ARG, "parameter value must be finite");
        const bool integral = (v == std::floor(v));
        switch (key) {
            case LBM_P_STORE:
                if (b->h) return bfail(b, LBM_E_STATE, "the store format is fixed once storage is bound");
                if (!integral || v < 0 || v > 3) return bfail(b, LBM_E_ARG, "store must be 0..3");
                b->store = (int)v;
                for (lbm_ctx* c : b->inst) c->store = b->store;
                break;
            case LBM_P_TILE_ODD:
            case LBM_P_TILE_EVEN: {
                if (!integral || !tile_ok((int)v)) return bfail(b, LBM_E_ARG, "tile must be 64, 128, 256 or 512");
                int& tile = (key == LBM_P_TILE_ODD ? b->tile_odd : b->tile_even);
                const int old = tile;
                tile = (int)v;
                if (!batch_shapes_fit(b)) {
                    tile = old;
                    return bfail(b, LBM_E_STATE, "blocks of several rows need the plain layout of an instance's state");
                }
                break;
            }
            case LBM_P_VECTOR: {
                if (!integral || v < 0 || v > 4) return bfail(b, LBM_E_ARG, "cells per thread must be 0, 1, 2 or 4");
                const int old = b->vw_req;
                b->vw_req = (int)v;
                if (!batch_shapes_fit(b)) {
                    b->vw_req = old;
                    return bfail(b, LBM_E_STATE, "blocks of several rows need the plain layout of an instance's state");
                }
                break;
            }
            case LBM_P_ODD_ROWS:
                if (!integral || v < 0 || v > 2) return bfail(b, LBM_E_ARG, "odd-step mode must be 0, 1 or 2");
                b->odd_rows = (int)v;
                break;
            case LBM_P_SPREAD:
                if (!integral || v < -1 || v > 16 || (v > 0 && v < kXcdChunkLog2))
                    return bfail(b, LBM_E_ARG, "brick spreading is -1 (by store), 0 (off) or a chunk log2 in [5, 16]");
                for (lbm_ctx* c : b->inst) c->spread = (int)v;
                break;
            case LBM_P_BRICK:
                if (b->initialized) return bfail(b, LBM_E_STATE, "the population layout is fixed once the state is initialised");
                if (!integral || v < 0 || v > (1 << 30)) return bfail(b, LBM_E_ARG, "rows per brick must be an integer >= 0");
                for (lbm_ctx* c : b->inst) c->brick_req = (int)v;
                break;
            case LBM_P_XCD_REMAP:
                if (v != 0.0 && v != 1.0) return bfail(b, LBM_E_ARG, "XCD remap is 0 or 1");
                b->xcd_remap = (int)v;
                break;
            case LBM_P_GRAPH_STEPS:
                if (!integral || v < 0 || v > 4096) return bfail(b, LBM_E_ARG, "graph chunk must be an integer in [0, 4096]");
                b->graph_steps = (int)v;
                break;
            case LBM_P_Y1:
            case LBM_P_NEWTON_TOL:
            case LBM_P_NEWTON_MAXIT:
            case LBM_P_COLLISION:
            case LBM_P_MRT_S_E:
            case LBM_P_MRT_S_EPS:
            case LBM_P_MRT_S_Q:
            case LBM_P_MRT_S_PI:
            case LBM_P_MRT_S_M:
            case LBM_P_VD_APLUS:
            case LBM_P_VD_UTAU:
                for (lbm_ctx* c : b->inst) {
                    c->batch_member = false;
                    int st = lbm_set_param(c, key, v);
                    c->batch_member = (b->h != nullptr);
                    if (st != LBM_OK) return bfail(b, st, c->err);
                }
                break;
            default:
                return bfail(b, LBM_E_ARG, "unknown or per-instance parameter key");
        }
        b->tables_ready = false;
        batch_drop_graphs(b);
        return LBM_OK;
    });
}

int lbm_batch_required_bytes(const lbm_batch* b, size_t* bytes)
{
    return bguard(const_cast<lbm_batch*>(b), [&]() -> int {
        if (!b || !bytes) return bfail(nullptr, LBM_E_ARG, "null argument");
        size_t total = 0;
        for (const lbm_ctx* c : b->inst) {
            size_t s = 0;
            lbm_required_bytes(c, &s);
            total += align256(s);
        }
        *bytes = total;
        return LBM_OK;
    });
}

int lbm_batch_bind_storage(lbm_batch* b, void* ptr, size_t bytes)
{
    return bguard(b, [&]() -> int {
        if (!b || !ptr) return bfail(b, LBM_E_ARG, "null argument");
        size_t need = 0;
        lbm_batch_required_bytes(b, &need);
        if (bytes < need) return bfail(b, LBM_E_ARG, "storage too small: need " + std::to_string(need) + " bytes");
        if (((uintptr_t)ptr) % 256 != 0) return bfail(b, LBM_E_ARG, "storage must be 256-byte aligned");
        b->offset.clear();
        size_t off = 0;
        for (lbm_ctx* c : b->inst) {
            size_t s = 0;
            lbm_required_bytes(c, &s);
            c->batch_member = false;
            int st = lbm_bind_storage(c, (char*)ptr + off, s);
            c->batch_member = true;
            if (st != LBM_OK) return bfail(b, st, c->err);
            c->stream = b->stream;
            b->offset.push_back(off);
            off += align256(s);
        }
        b->dev = b->inst[0]->dev;
        b->h = ptr;
        b->bytes = bytes;
        b->initialized = false;
        b->tables_ready = false;
        batch_drop_graphs(b);
        return LBM_OK;
    });
}

int lbm_batch_set_stream(lbm_batch* b, void* s)
{
    return bguard(b, [&]() -> int {
        if (!b) return bfail(nullptr, LBM_E_ARG, "null batch");
        b->stream = (hipStream_t)s;
        for (lbm_ctx* c : b->inst) c->stream = b->stream;
        return LBM_OK;
    });
}

int lbm_batch_init_spalding(lbm_batch* b, const double* u_tau, double noise, const uint64_t* seeds)
{
    return bguard(b, [&]() -> int {
        if (!b || !u_tau || !seeds) return bfail(b, LBM_E_ARG, "null argument");
        if (!b->h) return bfail(b, LBM_E_STATE, "no storage bound");
        DeviceGuard dg(b->dev);
        batch_apply_shapes(b);  // the instances' layouts follow the shapes they will run with
        for (int i = 0; i < b->n; ++i) {
            int st = init_spalding_impl(b->inst[i], u_tau[i], noise, seeds[i]);
            if (st != LBM_OK) return bfail(b, st, "instance " + std::to_string(i) + ": " + b->inst[i]->err);
        }
        b->steps = 0;
        b->layout_s = 0;
        b->initialized = true;
        return LBM_OK;
    });
}

int lbm_batch_step(lbm_batch* b, int64_t n)
{
    return bguard(b, [&]() -> int {
        if (!b) return bfail(nullptr, LBM_E_ARG, "null batch");
        if (!b->h || !b->initialized) return bfail(b, LBM_E_STATE, "batch not bound and initialised");
        if (n < 0) return bfail(b, LBM_E_ARG, "n must be >= 0");
        if (n == 0) return LBM_OK;
        DeviceGuard dg(b->dev);
        int st = batch_tables(b);
        if (st != LBM_OK) return st;
        for (lbm_ctx* c : b->inst)
            if ((st = refresh_damping(c, b->stream)) != LBM_OK) return bfail(b, st, c->err);
        long long left = n;
        while (left > 0) {
            if (b->graph_steps > 0 && left >= b->graph_steps) {
                const long long L = b->graph_steps;
                GraphKey key{b->layout_s, (int)L, 0, 0};
                auto it = b->graphs.find(key);
                if (it == b->graphs.end()) {
                    if (!b->cap_stream) LBM_BHIP(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
                    hipGraph_t g = nullptr;
                    LBM_BHIP(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
                    hipError_t e = batch_enqueue(b, b->cap_stream, b->layout_s, L);
                    hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
                    if (e != hipSuccess || e2 != hipSuccess) {
                        if (g) (void)hipGraphDestroy(g);
                        return bfail(b, LBM_E_DEVICE, std::string("graph capture: ") +
                                                          hipGetErrorString(e != hipSuccess ? e : e2));
                    }
                    hipGraphExec_t ex = nullptr;
                    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(g);
                    if (e != hipSuccess) return bfail(b, LBM_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
                    try {
                        it = b->graphs.emplace(key, ex).first;
                    } catch (...) {
                        (void)hipGraphExecDestroy(ex);
                        throw;
                    }
                }
                LBM_BHIP(b, hipGraphLaunch(it->second, b->stream));
                batch_advance(b, L);
                left -= L;
            } else {
                LBM_BHIP(b, batch_enqueue(b, b->stream, b->layout_s, 1));
                batch_advance(b, 1);
                left -= 1;
            }
        }
        return LBM_OK;
    });
}

int lbm_batch_sync(lbm_batch* b, int64_t* first_bad_step, int32_t* first_bad_instance)
{
    return bguard(b, [&]() -> int {
        if (!b) return bfail(nullptr, LBM_E_ARG, "null batch");
        if (first_bad_step) *first_bad_step = -1;
        if (first_bad_instance) *first_bad_instance = -1;
        if (!b->h) return LBM_OK;
        DeviceGuard dg(b->dev);
        LBM_BHIP(b, hipStreamSynchronize(b->stream));
        int worst = LBM_OK;
        for (int i = 0; i < b->n; ++i) {
            int64_t fb = -1;
            int st = lbm_sync(b->inst[i], &fb);
            if (st == LBM_E_DEVICE) return bfail(b, st, b->inst[i]->err);
            if (st != LBM_OK && worst == LBM_OK) {
                worst = st;
                if (first_bad_step) *first_bad_step = fb;
                if (first_bad_instance) *first_bad_instance = i;
                b->err = "instance " + std::to_string(i) + ": " + b->inst[i]->err;
            }
        }
        return worst;
    });
}

lbm_ctx* lbm_batch_instance(lbm_batch* b, int32_t i)
{
    if (!b || i < 0 || i >= b->n) return nullptr;
    return b->inst[i];
}

int lbm_batch_autotune(lbm_batch* b, int steps, int32_t* tiles)
{
    return bguard(b, [&]() -> int {
        if (!b) return bfail(nullptr, LBM_E_ARG, "null batch");
        if (!b->h) return bfail(b, LBM_E_STATE, "no storage bound");
        if (b->initialized) return bfail(b, LBM_E_STATE, "autotune runs before the state is initialised");
        if (steps < 2) return bfail(b, LBM_E_ARG, "steps must be >= 2");
        DeviceGuard dg(b->dev);
        std::vector<double> ut(b->n);
        std::vector<uint64_t> seeds(b->n, 0);
        for (int i = 0; i < b->n; ++i) ut[i] = std::sqrt(std::fabs(b->inst[i]->fx) * b->inst[i]->ny * 0.5);
        int st = lbm_batch_init_spalding(b, ut.data(), 0.05, seeds.data());
        if (st != LBM_OK) return st;
        for (lbm_ctx* c : b->inst) c->initialized = false;  // timing states: layouts follow the candidates
        const int tcand[4] = {64, 128, 256, 512};
        const int vcand[3] = {1, 2, 4};
        TimingEvents tev;
        if (!tev.create()) return bfail(b, LBM_E_DEVICE, "autotune: event creation failed");
        hipEvent_t* ev = tev.ev;
        hipError_t err = hipSuccess;
        // mean odd and even step times (ms) of the current settings: one warm-up
        // pair, then steps / 2 timed pairs
        auto measure = [&](float* to, float* te) -> bool {
            b->tables_ready = false;
            if ((st = batch_tables(b)) != LBM_OK) return false;
            const int pairs = std::max(1, steps / 2);
            *to = *te = 0.f;
            for (int r = 0; r <= pairs && err == hipSuccess; ++r) {
                err = hipEventRecord(ev[0], b->stream);
                if (err == hipSuccess) err = batch_enqueue(b, b->stream, 0, 1);
                if (err == hipSuccess) err = hipEventRecord(ev[1], b->stream);
                if (err == hipSuccess) err = batch_enqueue(b, b->stream, 1, 1);
                if (err == hipSuccess) err = hipEventRecord(ev[2], b->stream);
                if (err == hipSuccess) err = hipEventSynchronize(ev[2]);
                float x = 0.f, y = 0.f;
                if (err == hipSuccess) err = hipEventElapsedTime(&x, ev[0], ev[1]);
                if (err == hipSuccess) err = hipEventElapsedTime(&y, ev[1], ev[2]);
                if (r > 0) {
                    *to += x / pairs;
                    *te += y / pairs;
                }
            }
            return err == hipSuccess;
        };
        // every cells-per-thread width with every block size (the odd and even
        // kernels timed apart, the width shared), then the odd step's row walk
        float best = 1e30f;
        int bo = b->tile_odd, be = b->tile_even, bv = batch_width(b);
        const int save_req = b->vw_req, save_rows = b->odd_rows;
        bool ok = true;
        for (int iv = 0; iv < 3 && ok; ++iv) {
            b->vw_req = vcand[iv];
            if (batch_width(b) != vcand[iv]) continue;
            float bo_t = 1e30f, be_t = 1e30f;
            int bo_k = 256, be_k = 256;
            for (int k = 0; k < 4 && ok; ++k) {
                b->tile_odd = b->tile_even = tcand[k];
                float to = 0.f, te = 0.f;
                if (!(ok = measure(&to, &te))) break;
                if (to < bo_t) { bo_t = to; bo_k = tcand[k]; }
                if (te < be_t) { be_t = te; be_k = tcand[k]; }
            }
            if (ok && bo_t + be_t < best) {
                best = bo_t + be_t;
                bo = bo_k;
                be = be_k;
                bv = vcand[iv];
            }
        }
        int brows = save_rows;
        if (ok) {
            b->vw_req = bv;
            b->tile_odd = bo;
            b->tile_even = be;
            float to0 = 0.f, te0 = 0.f;
            ok = measure(&to0, &te0);
            for (int m : {0, 2}) {
                if (!ok || m == save_rows) continue;
                b->odd_rows = m;
                float to = 0.f, te = 0.f;
                if (!(ok = measure(&to, &te))) break;
                if (to < to0 * 0.99f) {
                    to0 = to;
                    brows = m;
                }
            }
        }
        b->vw_req = ok ? bv : save_req;
        b->odd_rows = ok ? brows : save_rows;
        b->tile_odd = bo;
        b->tile_even = be;
        b->tables_ready = false;
        b->initialized = false;
        for (lbm_ctx* c : b->inst) c->initialized = false;
        batch_drop_graphs(b);
        if (st != LBM_OK) return st;
        if (err != hipSuccess) return bfail(b, LBM_E_DEVICE, std::string("autotune: ") + hipGetErrorString(err));
        if (tiles) {
            tiles[0] = bo;
            tiles[1] = be;
            tiles[2] = bv;
        }
        return LBM_OK;
    });
}

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : g_err.c_str(); }

}  // extern "C"
