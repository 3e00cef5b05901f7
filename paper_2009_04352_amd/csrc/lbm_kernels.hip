// Device kernels of the WFB LBM-LES channel step for CDNA4 (gfx950).
//
// Method: Han, Ooka & Kikumoto, "A wall function approach in lattice
// Boltzmann method" (arXiv 2009.04352).  One fused kernel per time step does,
// for every cell: streaming (Eq. 1) with wall reflections (bounce-back, Eq. 3
// in 3-D form; mirror reflection, Eq. 4 in 3-D form), the wall-function bounce
// correction at wall-adjacent cells (Eq. 13-17, Newton on Spalding's law in
// FP64), moments (Eq. 2), a Smagorinsky eddy viscosity from the local
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
#include <hip/hip_runtime.h>
#include <math.h>
#include <utility>

#include "lattice.h"
#include "lbm_internal.h"
#include "store.h"

namespace lbmwf {

// ------------------------------------------------------------- utilities

template <typename F, int... As>
__device__ __forceinline__ void for_each_dir_impl(F&& fn, std::integer_sequence<int, As...>)
{
    (fn(std::integral_constant<int, As>{}), ...);
}

// Calls fn(std::integral_constant<int, a>) for a = 0 .. 18 in order.
template <typename F>
__device__ __forceinline__ void for_each_dir(F&& fn)
{
    for_each_dir_impl(fn, std::make_integer_sequence<int, kQ>{});
}

// Tile of a block.  Blocks are dispatched round-robin over the 8 XCDs; the
// remap hands XCD k a contiguous range of tiles, so neighbouring x-tiles of
// a row (which share cache lines at their ends) meet in the same L2.
__device__ __forceinline__ int tile_of_block(int b, int ntiles, int remap)
{
    if (!remap) return b;
    const int q = ntiles >> 3, r = ntiles & 7;
    const int k = b & 7, j = b >> 3;
    return k * q + min(k, r) + j;
}

// splitmix64 (Steele, Lea & Flood 2014): output k of the generator seeded
// with `seed`.
__device__ __forceinline__ unsigned long long splitmix64_at(unsigned long long seed, unsigned long long k)
{
    unsigned long long z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double uniform01(unsigned long long seed, unsigned long long k)
{
    return (double)(splitmix64_at(seed, k) >> 11) * (1.0 / 9007199254740992.0);
}

// ------------------------------------------------------ wall function (FP64)

// Friction velocity from Spalding's law (Eq. 16-17).  In p = u+ = U / u_tau
// with R = y1 U / nu the law reads H(p) = p Sp(p) - R = 0; Newton from the
// viscous-sublayer guess p0 = sqrt(R) decreases monotonically to the root
// because H is increasing and convex with H(p0) >= 0.
__device__ __forceinline__ double wall_utau(double U, double y1, double nu, double kappa, double ekb, double tol,
                                            int maxit, int& iters, bool& fail)
{
    const double R = y1 * U / nu;
    double p = sqrt(R);
    iters = 0;
    fail = true;
    for (int it = 1; it <= maxit; ++it) {
        const double k = kappa * p;
        const double ek = exp(k);
        const double k2 = 0.5 * k * k;
        const double br = ek - 1.0 - k - k2;              // e^k - 1 - k - k^2/2
        const double sp = p + ekb * (br - k2 * k * (1.0 / 3.0));
        const double dsp = 1.0 + kappa * ekb * br;
        const double pn = p - (p * sp - R) / (sp + p * dsp);
        iters = it;
        if (fabs(pn - p) <= tol * pn) {
            p = pn;
            fail = false;
            break;
        }
        p = pn;
    }
    return U / p;
}

struct WallRecord {
    double taux, tauz, utau, U;
};

// WFB correction of the gathered (free-slip) populations of one wall cell:
// tau_w from the wall function, split along the wall-parallel velocity
// (Eq. 15) and added as +-tau/2 to the four reflected diagonal populations
// (Eq. 13-14 with dt = dy = 1).  Top wall: the bottom rule mirrored in y.
template <typename R>
__device__ __forceinline__ WallRecord wfb_correct(R (&f)[kQ], bool top, double fx, double y1, double nu0,
                                                  double kappa, double ekb, double tol, int maxit, int& iters,
                                                  bool& fail)
{
    R drho = R(0), jx = R(0), jz = R(0);
    for_each_dir([&](auto A) {
        constexpr int a = decltype(A)::value;
        drho += f[a];
        if constexpr (kEx[a] == 1) jx += f[a];
        if constexpr (kEx[a] == -1) jx -= f[a];
        if constexpr (kEz[a] == 1) jz += f[a];
        if constexpr (kEz[a] == -1) jz -= f[a];
    });
    const R rho = R(1) + drho;
    const double vx = (double)((jx + R(0.5) * (R)fx) / rho);
    const double vz = (double)(jz / rho);
    const double U = sqrt(vx * vx + vz * vz);
    WallRecord rec{0.0, 0.0, 0.0, U};
    iters = 0;
    fail = false;
    if (U > 0.0) {
        const double ut = wall_utau(U, y1, nu0, kappa, ekb, tol, maxit, iters, fail);
        const double tauw = (double)rho * ut * ut;
        rec.taux = -(vx / U) * tauw;
        rec.tauz = -(vz / U) * tauw;
        rec.utau = ut;
    }
    const R hx = (R)(0.5 * rec.taux), hz = (R)(0.5 * rec.tauz);
    if (!top) {
        f[7] += hx;
        f[14] -= hx;
        f[11] += hz;
        f[17] -= hz;
    } else {
        f[mirror_y(7)] += hx;
        f[mirror_y(14)] -= hx;
        f[mirror_y(11)] += hz;
        f[mirror_y(17)] -= hz;
    }
    return rec;
}

// ------------------------------------------------- collision (Sec. 3.1, Eq. 1)

// The library is compiled without automatic contraction, so that every
// kernel evaluates the same operations in the same order (odd and even steps,
// single and batched launches agree bit for bit); fused multiply-adds are
// written out where they are wanted.
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename R>
struct Moments {
    R rho, ux, uy, uz;
};

// Moments (Eq. 2, half-force shift), Smagorinsky relaxation time from the
// non-equilibrium stress, BGK towards the second-order equilibrium and the
// Guo force term, in place on h = f - w.
template <typename R>
__device__ __forceinline__ Moments<R> collide(R (&f)[kQ], R tau0, R cs2_18, R fx)
{
    R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
    R sxx = R(0), syy = R(0), szz = R(0), sxy = R(0), sxz = R(0), syz = R(0);
    for_each_dir([&](auto A) {
        constexpr int a = decltype(A)::value;
        const R v = f[a];
        drho += v;
        if constexpr (kEx[a] == 1) jx += v;
        if constexpr (kEx[a] == -1) jx -= v;
        if constexpr (kEy[a] == 1) jy += v;
        if constexpr (kEy[a] == -1) jy -= v;
        if constexpr (kEz[a] == 1) jz += v;
        if constexpr (kEz[a] == -1) jz -= v;
        if constexpr (kEx[a] != 0) sxx += v;
        if constexpr (kEy[a] != 0) syy += v;
        if constexpr (kEz[a] != 0) szz += v;
        if constexpr (kEx[a] * kEy[a] == 1) sxy += v;
        if constexpr (kEx[a] * kEy[a] == -1) sxy -= v;
        if constexpr (kEx[a] * kEz[a] == 1) sxz += v;
        if constexpr (kEx[a] * kEz[a] == -1) sxz -= v;
        if constexpr (kEy[a] * kEz[a] == 1) syz += v;
        if constexpr (kEy[a] * kEz[a] == -1) syz -= v;
    });
    const R rho = R(1) + drho;
    const R inv = R(1) / rho;
    const R ux = fmad(R(0.5), fx, jx) * inv, uy = jy * inv, uz = jz * inv;
    // Pi_neq = sum e e h - sum e e h_eq, with sum e e h_eq = drho/3 I + rho u u
    const R c3 = drho * R(1.0 / 3.0);
    const R rux = rho * ux, ruy = rho * uy;
    const R pxx = fmad(-rux, ux, sxx - c3), pyy = fmad(-ruy, uy, syy - c3), pzz = fmad(-rho * uz, uz, szz - c3);
    const R pxy = fmad(-rux, uy, sxy), pxz = fmad(-rux, uz, sxz), pyz = fmad(-ruy, uz, syz);
    const R offd = fmad(pxy, pxy, fmad(pxz, pxz, pyz * pyz));
    const R pp = fmad(pxx, pxx, fmad(pyy, pyy, fmad(pzz, pzz, R(2) * offd)));
    const R qn = sqrt(R(2) * pp);
    const R taue = R(0.5) * (tau0 + sqrt(fmad(tau0, tau0, cs2_18 * qn * inv)));
    const R om = R(1) / taue;
    const R fc = fmad(R(-0.5), om, R(1)) * fx;  // (1 - 1/(2 tau_e)) Fx
    const R usq = R(1.5) * fmad(ux, ux, fmad(uy, uy, uz * uz));
    for_each_dir([&](auto A) {
        constexpr int a = decltype(A)::value;
        R eu = R(0);
        if constexpr (kEx[a] == 1) eu += ux;
        if constexpr (kEx[a] == -1) eu -= ux;
        if constexpr (kEy[a] == 1) eu += uy;
        if constexpr (kEy[a] == -1) eu -= uy;
        if constexpr (kEz[a] == 1) eu += uz;
        if constexpr (kEz[a] == -1) eu -= uz;
        constexpr R w = weight<R>(a);
        const R t = fmad(eu, fmad(R(4.5), eu, R(3)), -usq);  // 3 e.u + 4.5 (e.u)^2 - 1.5 u.u
        const R heq = w * fmad(rho, t, drho);
        R force = R(-3) * ux;                                 // 3 (e - u) . F + 9 (e . u)(e . F), per unit Fx
        if constexpr (kEx[a] != 0) force += fmad(R(9 * kEx[a]), eu, R(3 * kEx[a]));
        f[a] = fmad(w * fc, force, fmad(-om, f[a] - heq, f[a]));
    });
    return Moments<R>{rho, ux, uy, uz};
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// --------------------------------------------------------- the fused step

constexpr int kMaxBlock = 512;

template <typename S, bool ODD, bool SPEC, bool WFB, bool STATS>
__global__ __launch_bounds__(kMaxBlock) void k_step(StepArgs p)
{
    using T = typename S::T;
    using R = typename S::R;
    T* __restrict__ h = (T*)p.h;
    const long long N = p.n;
    const int tile = tile_of_block(blockIdx.x, p.ntiles, p.xcd_remap);
    const int row = tile / p.ntx;
    const int xt = tile - row * p.ntx;
    const int y = row % p.ny;
    const int z = row / p.ny;
    const int x = xt * p.tile_x + (int)threadIdx.x;
    const bool active = x < p.nx;
    const bool bot = (y == 0), top = (y == p.ny - 1);  // uniform over the block

    const unsigned nx = (unsigned)p.nx, ny = (unsigned)p.ny;
    const unsigned xm = (x == 0) ? nx - 1 : (unsigned)x - 1;
    const unsigned xp = (x == p.nx - 1) ? 0u : (unsigned)x + 1;
    const unsigned zm = (z == 0) ? (unsigned)p.nz - 1 : (unsigned)z - 1;
    const unsigned zp = (z == p.nz - 1) ? 0u : (unsigned)z + 1;
    // cell offset of (x + dx, y + dy, z + dz), x and z periodic; dy must stay inside
    auto off = [&](int dx, int dy, int dz) -> unsigned {
        const unsigned xx = dx < 0 ? xm : (dx > 0 ? xp : (unsigned)x);
        const unsigned zz = dz < 0 ? zm : (dz > 0 ? zp : (unsigned)z);
        return xx + nx * ((unsigned)(y + dy) + ny * zz);
    };

    R f[kQ];
    Moments<R> m{R(1), R(0), R(0), R(0)};
    int iters = 0;
    if (active) {
        // a1/a2: gather (odd: pull from neighbours with wall reflections; even: own slots)
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            constexpr int ex = kEx[a], ey = kEy[a], ez = kEz[a];
            if constexpr (ODD) {
                const bool from_wall = (ey == 1 && bot) || (ey == -1 && top);
                if (from_wall) {
                    if constexpr (!SPEC || !is_tangential(a))
                        f[a] = S::load(h + (long long)a * N + off(0, 0, 0));
                    else
                        f[a] = S::load(h + (long long)opp(mirror_y(a)) * N + off(-ex, 0, -ez));
                } else {
                    f[a] = S::load(h + (long long)opp(a) * N + off(-ex, -ey, -ez));
                }
            } else {
                f[a] = S::load(h + (long long)a * N + off(0, 0, 0));
            }
        });
        // a3: wall-function bounce at wall-adjacent cells (wave-uniform branch)
        if constexpr (WFB) {
            if (bot || top) {
                bool fail = false;
                wfb_correct<R>(f, top, p.fx, p.y1, p.nu0, p.kappa, p.ekb, p.newton_tol, p.newton_maxit, iters, fail);
                if (fail) {
                    atomicOr(&p.flags->status, 2);
                    atomicMin(&p.flags->first_bad, (unsigned long long)p.flags->cnt[ODD ? 1 : 0]);
                }
            }
        }
        // a4-a6: moments, Smagorinsky, BGK + body force
        m = collide<R>(f, (R)p.tau0, (R)p.cs2_18, (R)p.fx);
        if (!(m.rho > R(0)) || !(m.rho < R(INFINITY))) {
            atomicOr(&p.flags->status, 1);
            atomicMin(&p.flags->first_bad, (unsigned long long)p.flags->cnt[ODD ? 1 : 0]);
        }
        // a7: store (odd: push to neighbours with wall reflections; even: own opposite slots)
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            constexpr int ex = kEx[a], ey = kEy[a], ez = kEz[a];
            if constexpr (ODD) {
                const bool to_wall = (ey == -1 && bot) || (ey == 1 && top);
                if (to_wall) {
                    if constexpr (!SPEC || !is_tangential(a))
                        S::store(h + (long long)opp(a) * N + off(0, 0, 0), f[a]);
                    else
                        S::store(h + (long long)mirror_y(a) * N + off(ex, 0, ez), f[a]);
                } else {
                    S::store(h + (long long)a * N + off(ex, ey, ez), f[a]);
                }
            } else {
                S::store(h + (long long)opp(a) * N + off(0, 0, 0), f[a]);
            }
        });
    }
    if constexpr (WFB) {
        if (bot || top) {
            const int mx = wave_max(iters);
            if ((threadIdx.x & 63) == 0 && mx > 0) atomicMax(&p.flags->max_newton_iters, mx);
        }
    }
    // a8: plane statistics of the sampled velocity, FP64, fixed order
    if constexpr (STATS) {
        __shared__ double red[kMaxBlock / 64][7];
        double v[7];
        const double ux = active ? (double)m.ux : 0.0, uy = active ? (double)m.uy : 0.0,
                     uz = active ? (double)m.uz : 0.0;
        v[0] = ux; v[1] = uy; v[2] = uz;
        v[3] = ux * ux; v[4] = uy * uy; v[5] = uz * uz; v[6] = ux * uy;
        const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            const double s = wave_sum(v[k]);
            if (ln == 0) red[wv][k] = s;
        }
        __syncthreads();
        if (threadIdx.x < 7) {
            double s = 0.0;
            const int nw = (blockDim.x + 63) >> 6;
            for (int w = 0; w < nw; ++w) s += red[w][threadIdx.x];
            p.partials[(long long)tile * 7 + threadIdx.x] = s;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) p.flags->cnt[ODD ? 0 : 1] = p.flags->cnt[ODD ? 1 : 0] + 1;
}

template <typename S, bool ODD>
static hipError_t launch_step_bc(int bc, bool stats, const StepArgs& a, hipStream_t s)
{
    const dim3 grid((unsigned)a.ntiles), block((unsigned)a.tile_x);
#define LBM_STEP(SPEC, WFB)                                                                     \
    do {                                                                                        \
        if (stats)                                                                              \
            hipLaunchKernelGGL((k_step<S, ODD, SPEC, WFB, true>), grid, block, 0, s, a);        \
        else                                                                                    \
            hipLaunchKernelGGL((k_step<S, ODD, SPEC, WFB, false>), grid, block, 0, s, a);       \
    } while (0)
    if (bc == kBB) LBM_STEP(false, false);
    else if (bc == kWFB) LBM_STEP(true, true);
    else LBM_STEP(true, false);
#undef LBM_STEP
    return hipGetLastError();
}

template <typename S>
static hipError_t launch_step_s(bool odd, int bc, bool stats, const StepArgs& a, hipStream_t s)
{
    return odd ? launch_step_bc<S, true>(bc, stats, a, s) : launch_step_bc<S, false>(bc, stats, a, s);
}

hipError_t launch_step(int store, bool odd, int bc, bool stats, const StepArgs& a, hipStream_t s)
{
    if (a.tile_x < 1 || a.tile_x > kMaxBlock || a.ntiles < 1) return hipErrorInvalidValue;
    switch (store) {
        case kStoreF64: return launch_step_s<StoreF64>(odd, bc, stats, a, s);
        case kStoreF32: return launch_step_s<StoreF32>(odd, bc, stats, a, s);
        case kStoreF16: return launch_step_s<StoreF16>(odd, bc, stats, a, s);
        case kStoreBF16: return launch_step_s<StoreBF16>(odd, bc, stats, a, s);
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
__global__ __launch_bounds__(256) void k_init(void* hv, long long n, int nx, int ny, const double* __restrict__ prof,
                                              double noise, unsigned long long seed)
{
    using T = typename S::T;
    T* h = (T*)hv;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int y = (int)((c / nx) % ny);
    const double up = prof[y];
    double d[3];
    for (int i = 0; i < 3; ++i) d[i] = noise * (2.0 * uniform01(seed, 3ull * (unsigned long long)c + i) - 1.0);
    const double ux = up * (1.0 + d[0]), uy = up * d[1], uz = up * d[2];
    const double usq = 1.5 * (ux * ux + uy * uy + uz * uz);
    for_each_dir([&](auto A) {
        constexpr int a = decltype(A)::value;
        const double eu = kEx[a] * ux + kEy[a] * uy + kEz[a] * uz;
        const double heq = weight<double>(a) * (3.0 * eu + 4.5 * eu * eu - usq);
        h[(long long)opp(a) * n + c] = S::from_double(heq);
    });
}

// ------------------------------------------------- state in canonical form

// in[a][i]: h of the post-collision f*_a(c), c = first + i; written in layout P.
template <typename S>
__global__ __launch_bounds__(256) void k_set_state(void* hv, long long n, long long first, long long count,
                                                   const double* __restrict__ in)
{
    using T = typename S::T;
    T* h = (T*)hv;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const long long c = first + i;
    for (int a = 0; a < kQ; ++a) h[(long long)opp(a) * n + c] = S::from_double(in[(long long)a * count + i]);
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

__device__ __forceinline__ long long cell_at(int x, int y, int z, int nx, int ny, int nz)
{
    x = (x % nx + nx) % nx;
    z = (z % nz + nz) % nz;
    return (long long)x + (long long)nx * ((long long)y + (long long)ny * z);
}

// out[a][i]: h of f*_a at cell i of the list (or first + i), from either layout.
template <typename S>
__global__ __launch_bounds__(256) void k_get_state(const void* hv, long long n, int nx, int ny, int nz, int layout_s,
                                                   int layout_spec, const long long* __restrict__ cells,
                                                   long long first, long long count, double* __restrict__ out)
{
    using T = typename S::T;
    const T* h = (const T*)hv;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const long long c = cells ? cells[i] : first + i;
    const Pos q = cell_pos(c, nx, ny);
    for_each_dir([&](auto A) {
        constexpr int a = decltype(A)::value;
        long long src;
        int slot;
        if (!layout_s) {
            slot = opp(a);
            src = c;
        } else {
            const int dy = q.y + kEy[a];
            if (dy >= 0 && dy < ny) {
                slot = a;
                src = cell_at(q.x + kEx[a], dy, q.z + kEz[a], nx, ny, nz);
            } else if (!layout_spec || !is_tangential(a)) {
                slot = opp(a);
                src = c;
            } else {
                slot = mirror_y(a);
                src = cell_at(q.x + kEx[a], q.y, q.z + kEz[a], nx, ny, nz);
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
        c = p.cells ? p.cells[i] : p.first + i;
        const Pos q = cell_pos(c, p.nx, p.ny);
        x = q.x; y = q.y; z = q.z;
    } else {
        const long long per = (long long)p.nx * p.nz;
        const int w = (int)(i / per);
        z = (int)((i % per) / p.nx);
        x = (int)(i % p.nx);
        y = w ? p.ny - 1 : 0;
        c = (long long)x + (long long)p.nx * ((long long)y + (long long)p.ny * z);
    }
    const bool bot = (y == 0), top = (y == p.ny - 1);
    const long long n = p.n;
    R f[kQ];
    for_each_dir([&](auto A) {
        constexpr int a = decltype(A)::value;
        constexpr int ex = kEx[a], ey = kEy[a], ez = kEz[a];
        if (p.layout_s) {
            f[a] = S::load(h + (long long)a * n + c);
        } else {
            const int sy = y - ey;
            if (sy >= 0 && sy < p.ny) {
                f[a] = S::load(h + (long long)opp(a) * n + cell_at(x - ex, sy, z - ez, p.nx, p.ny, p.nz));
            } else if (p.bc == kBB || !is_tangential(a)) {
                f[a] = S::load(h + (long long)a * n + c);
            } else {
                f[a] = S::load(h + (long long)opp(mirror_y(a)) * n + cell_at(x - ex, y, z - ez, p.nx, p.ny, p.nz));
            }
        }
    });
    WallRecord rec{0.0, 0.0, 0.0, 0.0};
    int iters = 0;
    if (p.bc == kWFB && (bot || top)) {
        bool fail = false;
        rec = wfb_correct<R>(f, top, p.fx, p.y1, p.nu0, p.kappa, p.ekb, p.newton_tol, p.newton_maxit, iters, fail);
        if (fail) iters = -iters;
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
        double* o = p.out + 4 * i;
        o[0] = (double)rho; o[1] = (double)ux; o[2] = (double)uy; o[3] = (double)uz;
        return;
    }
    if (p.bc == kBB) {
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
    double* o = p.out + 4 * i;
    o[0] = rec.taux; o[1] = rec.tauz; o[2] = rec.utau; o[3] = rec.U;
    if (p.iters) p.iters[i] = iters;
}

// --------------------------------------------- re-reflection of a layout S

// When the boundary switches between bounce-back and mirror reflection after
// an odd number of steps, the wall-crossing populations already reflected by
// the old rule are moved to where the new rule puts them.  Pass 0 gathers the
// five outgoing populations of every wall cell into tmp, pass 1 scatters them.
template <typename S>
__global__ __launch_bounds__(256) void k_relayout(void* hv, long long n, int nx, int ny, int nz, int from_spec,
                                                  int to_spec, double* __restrict__ tmp, int pass)
{
    using T = typename S::T;
    T* h = (T*)hv;
    const long long per = (long long)nx * nz;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * per) return;
    const int w = (int)(i / per);
    const int z = (int)((i % per) / nx), x = (int)(i % nx);
    const int y = w ? ny - 1 : 0;
    const long long c = (long long)x + (long long)nx * ((long long)y + (long long)ny * z);
    const int spec = pass == 0 ? from_spec : to_spec;
    int k = 0;
    for_each_dir([&](auto A) {
        constexpr int b = decltype(A)::value;
        if ((w == 0 && kEy[b] == -1) || (w == 1 && kEy[b] == 1)) {
            long long slot;
            if (!spec || !is_tangential(b))
                slot = (long long)opp(b) * n + c;
            else
                slot = (long long)mirror_y(b) * n + cell_at(x + kEx[b], y, z + kEz[b], nx, ny, nz);
            if (pass == 0)
                tmp[i * 5 + k] = S::to_double(h[slot]);
            else
                h[slot] = S::from_double(tmp[i * 5 + k]);
            ++k;
        }
    });
}

// ----------------------------------------------------------- misc kernels

__global__ __launch_bounds__(256) void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, long long n)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_wall_utau(const double* __restrict__ U, int n, double y1, double nu,
                                                   double kappa, double ekb, double tol, int maxit,
                                                   double* __restrict__ ut, int* __restrict__ iters)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int it = 0;
    bool fail = false;
    double r = 0.0;
    if (U[i] > 0.0) r = wall_utau(U[i], y1, nu, kappa, ekb, tol, maxit, it, fail);
    ut[i] = fail ? -1.0 : r;
    iters[i] = it;
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
template <typename S> struct GetK { static constexpr auto fn = k_get_state<S>; };
template <typename S> struct ObsK { static constexpr auto fn = k_observe<S>; };
template <typename S> struct RelK { static constexpr auto fn = k_relayout<S>; };

static dim3 blocks_for(long long n, int bs) { return dim3((unsigned)((n + bs - 1) / bs)); }

hipError_t launch_init_spalding(int store, void* h, long long n, int nx, int ny, int nz, const double* profile,
                                double noise, unsigned long long seed, hipStream_t s)
{
    (void)nz;
    if (n <= 0) return hipSuccess;
    return dispatch_store<InitK>(store, blocks_for(n, 256), dim3(256), s, h, n, nx, ny, profile, noise, seed);
}

hipError_t launch_set_state(int store, void* h, long long n, long long first, long long count, const double* in,
                            hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    return dispatch_store<SetK>(store, blocks_for(count, 256), dim3(256), s, h, n, first, count, in);
}

hipError_t launch_get_state(int store, const void* h, long long n, int nx, int ny, int nz, int layout_s,
                            int layout_spec, const long long* cells, long long first, long long count, double* out,
                            hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    return dispatch_store<GetK>(store, blocks_for(count, 256), dim3(256), s, h, n, nx, ny, nz, layout_s, layout_spec,
                                cells, first, count, out);
}

hipError_t launch_observe(int store, const ObsArgs& a, hipStream_t s)
{
    if (a.count <= 0) return hipSuccess;
    return dispatch_store<ObsK>(store, blocks_for(a.count, 256), dim3(256), s, a);
}

hipError_t launch_relayout(int store, void* h, long long n, int nx, int ny, int nz, int from_spec, int to_spec,
                           double* tmp, hipStream_t s)
{
    const long long m = 2ll * nx * nz;
    hipError_t e = dispatch_store<RelK>(store, blocks_for(m, 256), dim3(256), s, h, n, nx, ny, nz, from_spec,
                                        to_spec, tmp, 0);
    if (e != hipSuccess) return e;
    return dispatch_store<RelK>(store, blocks_for(m, 256), dim3(256), s, h, n, nx, ny, nz, from_spec, to_spec, tmp,
                                1);
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s)
{
    if (bytes % 16 != 0) return hipErrorInvalidValue;
    const long long n = (long long)(bytes / 16);
    if (n == 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 256 * 1024) blocks = 256 * 1024;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, (const uint4*)src, (uint4*)dst, n);
    return hipGetLastError();
}

hipError_t launch_wall_utau(const double* U, int n, double y1, double nu, double kappa, double bconst, double tol,
                            int maxit, double* utau, int* iters, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_wall_utau, blocks_for(n, 256), dim3(256), 0, s, U, n, y1, nu, kappa, exp(-kappa * bconst),
                       tol, maxit, utau, iters);
    return hipGetLastError();
}

}  // namespace lbmwf
