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

// Reciprocal and square root: one hardware instruction in FP32 (about one ulp),
// the IEEE operations in FP64.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float sqrt_r(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }

// The pairs (a, a + 1) of opposite directions, a odd, used below with these
// velocities (Table A-1).
static_assert(kEx[1] == 1 && kEy[3] == 1 && kEz[5] == 1, "axis pairs");
static_assert(kEx[7] == 1 && kEy[7] == 1 && kEz[7] == 0, "pair 7");
static_assert(kEx[9] == 1 && kEy[9] == 0 && kEz[9] == 1, "pair 9");
static_assert(kEx[11] == 0 && kEy[11] == 1 && kEz[11] == 1, "pair 11");
static_assert(kEx[13] == 1 && kEy[13] == -1 && kEz[13] == 0, "pair 13");
static_assert(kEx[15] == 1 && kEy[15] == 0 && kEz[15] == -1, "pair 15");
static_assert(kEx[17] == 0 && kEy[17] == 1 && kEz[17] == -1, "pair 17");

// Moments (Eq. 2, half-force shift), Smagorinsky relaxation time from the
// non-equilibrium stress, BGK towards the second-order equilibrium and the
// Guo force term, in place on h = f - w.  Opposite directions are handled as
// pairs: with s = h_a + h_b and d = h_a - h_b the moments are sums of s or d,
// the equilibrium splits into an even part w (drho + rho (4.5 (e.u)^2 - 1.5 u.u))
// and an odd part 3 w rho e.u, and the force term into -3 u_x + 9 e_x e.u and
// 3 e_x (per unit force along x).
template <typename R>
__device__ __forceinline__ Moments<R> collide(R (&f)[kQ], R tau0, R cs2_18, R fx)
{
    R s[kQ], d[kQ];  // indexed by the odd member of each pair
    R drho = f[0];
    for_each_dir([&](auto A) {
        constexpr int a = decltype(A)::value;
        if constexpr (a % 2 == 1) {
            s[a] = f[a] + f[a + 1];
            d[a] = f[a] - f[a + 1];
            drho += s[a];
        }
    });
    const R jx = ((d[1] + d[7]) + (d[9] + d[13])) + d[15];
    const R jy = ((d[3] + d[7]) + (d[11] - d[13])) + d[17];
    const R jz = ((d[5] + d[9]) + (d[11] - d[15])) - d[17];
    const R sxx = ((s[1] + s[7]) + (s[9] + s[13])) + s[15];
    const R syy = ((s[3] + s[7]) + (s[11] + s[13])) + s[17];
    const R szz = ((s[5] + s[9]) + (s[11] + s[15])) + s[17];
    const R sxy = s[7] - s[13], sxz = s[9] - s[15], syz = s[11] - s[17];

    const R rho = R(1) + drho;
    const R inv = rcp(rho);
    const R ux = fmad(R(0.5), fx, jx) * inv, uy = jy * inv, uz = jz * inv;
    // Pi_neq = sum e e h - sum e e h_eq, with sum e e h_eq = drho/3 I + rho u u
    const R c3 = drho * R(1.0 / 3.0);
    const R rux = rho * ux, ruy = rho * uy;
    const R pxx = fmad(-rux, ux, sxx - c3), pyy = fmad(-ruy, uy, syy - c3), pzz = fmad(-rho * uz, uz, szz - c3);
    const R pxy = fmad(-rux, uy, sxy), pxz = fmad(-rux, uz, sxz), pyz = fmad(-ruy, uz, syz);
    const R offd = fmad(pxy, pxy, fmad(pxz, pxz, pyz * pyz));
    const R pp = fmad(pxx, pxx, fmad(pyy, pyy, fmad(pzz, pzz, R(2) * offd)));
    const R qn = sqrt_r(R(2) * pp);
    const R taue = R(0.5) * (tau0 + sqrt_r(fmad(tau0, tau0, cs2_18 * qn * inv)));
    const R om = rcp(taue);
    const R omh = R(0.5) - R(0.5) * om;          // (1 - omega) / 2
    const R fc = fmad(R(-0.5), om, R(1)) * fx;   // (1 - 1/(2 tau_e)) Fx
    const R usq = R(1.5) * fmad(ux, ux, fmad(uy, uy, uz * uz));
    const R m3ux = R(-3) * ux;

    {   // rest population: e = 0
        constexpr R w = weight<R>(0);
        const R heq = w * fmad(rho, -usq, drho);
        f[0] = fmad(-om, f[0] - heq, f[0]) + (w * fc) * m3ux;
    }
    for_each_dir([&](auto A) {
        constexpr int a = decltype(A)::value;
        if constexpr (a % 2 == 1) {
            constexpr int ex = kEx[a];
            constexpr R w = weight<R>(a);
            R eu = R(0);
            if constexpr (kEx[a] == 1) eu = ux;
            if constexpr (kEy[a] == 1) eu = (kEx[a] != 0) ? eu + uy : uy;
            if constexpr (kEy[a] == -1) eu = eu - uy;
            if constexpr (kEz[a] == 1) eu = (kEx[a] != 0 || kEy[a] != 0) ? eu + uz : uz;
            if constexpr (kEz[a] == -1) eu = eu - uz;
            const R hs = w * fmad(rho, fmad(R(4.5) * eu, eu, -usq), drho);   // even part of h_eq
            const R hd = (R(3) * w) * rho * eu;                              // odd part of h_eq
            R fs = m3ux;                                                     // even part of the force term
            if constexpr (ex != 0) fs = fmad(R(9 * ex), eu, m3ux);
            fs = (w * fc) * fs;
            // half sum and half difference of the post-collision pair
            const R S = fmad(omh, s[a], fmad(om, hs, fs));
            R D;
            if constexpr (ex != 0) D = fmad(omh, d[a], fmad(om, hd, (w * fc) * R(3 * ex)));
            else D = fmad(omh, d[a], om * hd);
            f[a] = S + D;
            f[a + 1] = S - D;
        }
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

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// A group of V consecutive populations of one direction, G = V * sizeof(T)
// bytes (2, 4 or 8), held in the low bytes of a u32x2.  Groups that no other
// thread touches move with non-temporal loads and stores (every slot is read
// once and written once per step); single elements at tile edges, which
// neighbouring blocks share cache lines with, stay cached.
template <typename S, int V>
struct Lane {
    using T = typename S::T;
    using R = typename S::R;
    static constexpr int kBytes = (int)sizeof(T);
    static constexpr int G = V * kBytes;
    static_assert(G == 2 || G == 4 || G == 8, "a group is 2, 4 or 8 bytes");

    template <bool NT>
    __device__ __forceinline__ static u32x2 load(const T* p)
    {
        if constexpr (G == 8) {
            if constexpr (NT) return __builtin_nontemporal_load((const u32x2*)p);
            else return *(const u32x2*)p;
        } else if constexpr (G == 4) {
            if constexpr (NT) return u32x2{__builtin_nontemporal_load((const unsigned int*)p), 0u};
            else return u32x2{*(const unsigned int*)p, 0u};
        } else {
            if constexpr (NT) return u32x2{(unsigned int)__builtin_nontemporal_load((const unsigned short*)p), 0u};
            else return u32x2{(unsigned int)*(const unsigned short*)p, 0u};
        }
    }
    template <bool NT>
    __device__ __forceinline__ static void store(T* p, u32x2 v)
    {
        if constexpr (G == 8) {
            if constexpr (NT) __builtin_nontemporal_store(v, (u32x2*)p);
            else *(u32x2*)p = v;
        } else if constexpr (G == 4) {
            if constexpr (NT) __builtin_nontemporal_store(v.x, (unsigned int*)p);
            else *(unsigned int*)p = v.x;
        } else {
            if constexpr (NT) __builtin_nontemporal_store((unsigned short)v.x, (unsigned short*)p);
            else *(unsigned short*)p = (unsigned short)v.x;
        }
    }
    // raw bits of one element (element sizes 2 and 4; groups of V >= 2)
    __device__ __forceinline__ static unsigned int load_elem(const T* p)
    {
        if constexpr (kBytes == 4) return *(const unsigned int*)p;
        else return (unsigned int)*(const unsigned short*)p;
    }
    __device__ __forceinline__ static void store_elem(T* p, unsigned int b)
    {
        if constexpr (kBytes == 4) *(unsigned int*)p = b;
        else *(unsigned short*)p = (unsigned short)b;
    }
    __device__ __forceinline__ static unsigned int first(u32x2 v)
    {
        if constexpr (kBytes == 4) return v.x;
        else return v.x & 0xffffu;
    }
    __device__ __forceinline__ static unsigned int last(u32x2 v)
    {
        if constexpr (kBytes == 4) return v.y;
        else if constexpr (V == 4) return v.y >> 16;
        else return v.x >> 16;
    }
    // the group holding only element b, as its last (first) element
    __device__ __forceinline__ static u32x2 as_last(unsigned int b)
    {
        if constexpr (kBytes == 4) return u32x2{0u, b};
        else if constexpr (V == 4) return u32x2{0u, b << 16};
        else return u32x2{b << 16, 0u};
    }
    __device__ __forceinline__ static u32x2 as_first(unsigned int b) { return u32x2{b, 0u}; }
    // [p, e0 .. e(V-2)]
    __device__ __forceinline__ static u32x2 shift_in_left(u32x2 v, unsigned int p)
    {
        if constexpr (kBytes == 4) return u32x2{p, v.x};
        else if constexpr (V == 4) return u32x2{(v.x << 16) | p, (v.y << 16) | (v.x >> 16)};
        else return u32x2{(v.x << 16) | p, 0u};
    }
    // [e1 .. e(V-1), q]
    __device__ __forceinline__ static u32x2 shift_in_right(u32x2 v, unsigned int q)
    {
        if constexpr (kBytes == 4) return u32x2{v.y, q};
        else if constexpr (V == 4) return u32x2{(v.x >> 16) | (v.y << 16), (v.y >> 16) | (q << 16)};
        else return u32x2{(v.x >> 16) | (q << 16), 0u};
    }
    // elements 1 .. V-1 of the group at p (the first one belongs to another block)
    __device__ __forceinline__ static void store_tail(T* p, u32x2 v)
    {
        if constexpr (kBytes == 4) {
            *(unsigned int*)(p + 1) = v.y;
        } else if constexpr (V == 4) {
            *(unsigned short*)(p + 1) = (unsigned short)(v.x >> 16);
            *(unsigned int*)(p + 2) = v.y;
        } else {
            *(unsigned short*)(p + 1) = (unsigned short)(v.x >> 16);
        }
    }
    // elements 0 .. V-2 of the group at p (the last one belongs to another block)
    __device__ __forceinline__ static void store_head(T* p, u32x2 v)
    {
        if constexpr (kBytes == 4) {
            *(unsigned int*)p = v.x;
        } else if constexpr (V == 4) {
            *(unsigned int*)p = v.x;
            *(unsigned short*)(p + 2) = (unsigned short)(v.y & 0xffffu);
        } else {
            *(unsigned short*)p = (unsigned short)(v.x & 0xffffu);
        }
    }
    __device__ __forceinline__ static R get(u32x2 v, int k)
    {
        if constexpr (kBytes == 8) {
            return __hiloint2double((int)v.y, (int)v.x);
        } else if constexpr (kBytes == 4) {
            return __uint_as_float(k == 0 ? v.x : v.y);
        } else {
            const unsigned int word = (k < 2) ? v.x : v.y;
            const unsigned short b = (unsigned short)((k & 1) ? (word >> 16) : (word & 0xffffu));
            if constexpr (S::kind == kStoreBF16) return bf16_to_f32(b);
            else return (float)__builtin_bit_cast(_Float16, b);
        }
    }
    __device__ __forceinline__ static void set(u32x2& v, int k, R r)
    {
        if constexpr (kBytes == 8) {
            v.x = (unsigned int)__double2loint(r);
            v.y = (unsigned int)__double2hiint(r);
        } else if constexpr (kBytes == 4) {
            if (k == 0) v.x = __float_as_uint(r);
            else v.y = __float_as_uint(r);
        } else {
            unsigned short b;
            if constexpr (S::kind == kStoreBF16) b = __builtin_bit_cast(unsigned short, (__bf16)r);
            else b = __builtin_bit_cast(unsigned short, (_Float16)r);
            const unsigned int word = (k < 2) ? v.x : v.y;
            const unsigned int nw = (k & 1) ? ((word & 0xffffu) | ((unsigned int)b << 16)) : ((word & 0xffff0000u) | b);
            if (k < 2) v.x = nw;
            else v.y = nw;
        }
    }
};

// Cells x0 .. x0 + V - 1 of one x-row owned by one thread.
struct RowLanes {
    int x0, nx;
    bool active;
    __device__ __forceinline__ unsigned wrapx(int x) const
    {
        return (unsigned)(x < 0 ? x + nx : (x >= nx ? x - nx : x));
    }
};

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

// One element read straight from a row, placed as the last (first) element of a group.
template <typename S, int V>
__device__ __forceinline__ u32x2 halo_as_last(const typename S::T* row, unsigned x)
{
    using Ln = Lane<S, V>;
    if constexpr (V == 1) return Ln::template load<false>(row + x);
    else return Ln::as_last(Ln::load_elem(row + x));
}
template <typename S, int V>
__device__ __forceinline__ u32x2 halo_as_first(const typename S::T* row, unsigned x)
{
    using Ln = Lane<S, V>;
    if constexpr (V == 1) return Ln::template load<false>(row + x);
    else return Ln::as_first(Ln::load_elem(row + x));
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
// BATCH: the instance of the tile and its parameters come from tables.
template <typename S, int V, bool ODD, int BCT, bool STATS>
__global__ __launch_bounds__(kMaxBlock) void k_step(StepArgs p0, const StepArgs* __restrict__ table,
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
    const bool spec = BATCH ? (p.bc != kBB) : (BCT != kBB);
    const bool wfb = BATCH ? (p.bc == kWFB) : (BCT == kWFB);
    constexpr bool MAYBE_WFB = BATCH || BCT == kWFB;
    constexpr bool MAYBE_SPEC = BATCH || BCT != kBB;

    T* h = (T*)p.h;
    const long long N = p.n;
    const int t = (int)threadIdx.x;
    const int nthr = (int)blockDim.x;
    // tile -> (x segment, group of rows, z)
    const int xt = tile % p.ntx;
    const int rest = tile / p.ntx;
    const int yt = rest % p.nyt;
    const int z = rest / p.nyt;
    const bool whole = (p.ntx == 1);
    const int tpr = whole ? p.nx / V : nthr;        // threads per row segment
    const int r = t / tpr, tr = t - r * tpr;
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

    const unsigned nx = (unsigned)p.nx, ny = (unsigned)p.ny;
    const unsigned zm = (z == 0) ? (unsigned)p.nz - 1 : (unsigned)z - 1;
    const unsigned zp = (z == p.nz - 1) ? 0u : (unsigned)z + 1;
    // start of the x-row (y + dy, z + dz) of direction slot s; only formed for rows inside the channel
    auto rowp = [&](int s, int dy, int dz) -> T* {
        const unsigned zz = dz < 0 ? zm : (dz > 0 ? zp : (unsigned)z);
        return h + (long long)s * N + (long long)(nx * ((unsigned)(y + dy) + ny * zz));
    };
    auto ld = [&](const T* rw) -> u32x2 { return Ln::template load<true>(rw + L.x0); };
    auto st = [&](T* rw, u32x2 v) { Ln::template store<true>(rw + L.x0, v); };

    // a1/a2: gather.  Odd: pull from neighbours with wall reflections; even: own slots.
    u32x2 w[kQ];
    for_each_dir([&](auto A) {
        constexpr int a = decltype(A)::value;
        constexpr int ey = kEy[a], ez = kEz[a];
        w[a] = u32x2{0u, 0u};
        if (L.active) {
            if constexpr (ODD) {
                const bool from_wall = (ey == 1 && bot) || (ey == -1 && top);
                if (from_wall) {
                    if (MAYBE_SPEC && spec && is_tangential(a)) w[a] = ld(rowp(opp(mirror_y(a)), 0, -ez));
                    else w[a] = ld(rowp(a, 0, 0));
                } else {
                    w[a] = ld(rowp(opp(a), -ey, -ez));
                }
            } else {
                w[a] = ld(rowp(a, 0, 0));
            }
        }
    });
    if constexpr (ODD) {
        // the x-shifted groups hold cells x0 .. x0 + V - 1 of the source row; shift by -e_x
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            if constexpr (kEx[a] != 0) xbuf[xslot(a) * nthr + t] = w[a];
        });
        __syncthreads();
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            constexpr int ex = kEx[a], ey = kEy[a], ez = kEz[a];
            if constexpr (ex != 0) {
                const bool from_wall = (ey == 1 && bot) || (ey == -1 && top);
                const bool shifted = !from_wall || (MAYBE_SPEC && spec && is_tangential(a));
                if (shifted && L.active) {
                    const u32x2* xb = xbuf + xslot(a) * nthr;
                    if constexpr (ex == 1) {  // needs the element at x0 - 1
                        u32x2 nb;
                        if (tr > 0) nb = xb[t - 1];
                        else if (whole) nb = xb[tb + nact - 1];
                        else nb = halo_as_last<S, V>(from_wall ? rowp(opp(mirror_y(a)), 0, -ez) : rowp(opp(a), -ey, -ez),
                                                     L.wrapx(L.x0 - 1));
                        w[a] = join_left<S, V>(w[a], nb);
                    } else {                  // needs the element at x0 + V
                        u32x2 nb;
                        if (tr < nact - 1) nb = xb[t + 1];
                        else if (whole) nb = xb[tb];
                        else nb = halo_as_first<S, V>(from_wall ? rowp(opp(mirror_y(a)), 0, -ez) : rowp(opp(a), -ey, -ez),
                                                      L.wrapx(L.x0 + V));
                        w[a] = join_right<S, V>(w[a], nb);
                    }
                }
            }
        });
    }

    double sm[7] = {0, 0, 0, 0, 0, 0, 0};
    int iters = 0;
    bool bad = false, newton_fail = false;
#pragma unroll
    for (int k = 0; k < V; ++k) {
        R f[kQ];
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            f[a] = Ln::get(w[a], k);
        });
        // a3: wall-function bounce at wall-adjacent cells
        if constexpr (MAYBE_WFB) {
            if (wfb && (bot || top)) {
                int it = 0;
                bool fail = false;
                wfb_correct<R>(f, top, p.fx, p.y1, p.nu0, p.kappa, p.ekb, p.newton_tol, p.newton_maxit, it, fail);
                iters = max(iters, it);
                newton_fail = newton_fail || fail;
            }
        }
        // a4-a6: moments, Smagorinsky, BGK + body force
        const Moments<R> m = collide<R>(f, (R)p.tau0, (R)p.cs2_18, (R)p.fx);
        bad = bad || !(m.rho > R(0)) || !(m.rho < R(INFINITY));
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            Ln::set(w[a], k, f[a]);
        });
        if constexpr (STATS) {
            const double ux = (double)m.ux, uy = (double)m.uy, uz = (double)m.uz;
            sm[0] += ux; sm[1] += uy; sm[2] += uz;
            sm[3] += ux * ux; sm[4] += uy * uy; sm[5] += uz * uz; sm[6] += ux * uy;
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
                    st(rowp(opp(a), 0, 0), w[a]);  // bounce-back into the cell's own slot
                } else if constexpr (ex == 0) {
                    st(mirrored ? rowp(mirror_y(a), 0, ez) : rowp(a, ey, ez), w[a]);
                } else {
                    T* dst = mirrored ? rowp(mirror_y(a), 0, ez) : rowp(a, ey, ez);
                    const u32x2* xb = xbuf + xslot(a) * nthr;
                    if constexpr (ex == 1) {  // cell x goes to x + 1: the group at x0 starts with x0 - 1's value
                        if (tr > 0 || whole) {
                            st(dst, join_left<S, V>(w[a], xb[tr > 0 ? t - 1 : tb + nact - 1]));
                        } else {
                            if constexpr (V > 1) Ln::store_tail(dst + L.x0, Ln::shift_in_left(w[a], 0u));
                        }
                        if (!whole && tr == nact - 1) {
                            if constexpr (V == 1) Ln::template store<false>(dst + L.wrapx(L.x0 + 1), w[a]);
                            else Ln::store_elem(dst + L.wrapx(L.x0 + V), Ln::last(w[a]));
                        }
                    } else {                  // cell x goes to x - 1: the group at x0 ends with x0 + V's value
                        if (tr < nact - 1 || whole) {
                            st(dst, join_right<S, V>(w[a], xb[tr < nact - 1 ? t + 1 : tb]));
                        } else {
                            if constexpr (V > 1) Ln::store_head(dst + L.x0, Ln::shift_in_right(w[a], 0u));
                        }
                        if (!whole && tr == 0) {
                            if constexpr (V == 1) Ln::template store<false>(dst + L.wrapx(L.x0 - 1), w[a]);
                            else Ln::store_elem(dst + L.wrapx(L.x0 - 1), Ln::first(w[a]));
                        }
                    }
                }
            });
        }
    } else {
        if (L.active) {
            for_each_dir([&](auto A) {
                constexpr int a = decltype(A)::value;
                st(rowp(opp(a), 0, 0), w[a]);
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
static hipError_t launch_step_v(bool odd, int bc, const StepArgs& a, hipStream_t s)
{
    return odd ? launch_step_bc<S, V, true>(bc, a, s) : launch_step_bc<S, V, false>(bc, a, s);
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

// Dispatch on the group width: F = launch_step_v or launch_batch_v style callable.
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

void step_geometry(int nx, int ny, int nz, int tile_x, int vw, StepArgs& a)
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
}

static bool step_args_ok(int store, const StepArgs& a)
{
    if (a.tile_x < 64 || a.tile_x > kMaxBlock || (a.tile_x & 63) || a.ntiles < 1) return false;
    if (!step_vector_width_ok(store, a.nx, a.vw)) return false;
    StepArgs g = a;
    step_geometry(a.nx, a.ny, a.nz, a.tile_x, a.vw, g);
    return g.ntx == a.ntx && g.rpb == a.rpb && g.nyt == a.nyt && g.ntiles == a.ntiles;
}

hipError_t launch_step(int store, bool odd, int bc, const StepArgs& a, hipStream_t s)
{
    if (!step_args_ok(store, a)) return hipErrorInvalidValue;
    auto go = [&](auto St) -> hipError_t {
        using S = decltype(St);
        return with_width<S>(a.vw, [&](auto Vc) { return launch_step_v<S, decltype(Vc)::value>(odd, bc, a, s); });
    };
    switch (store) {
        case kStoreF64: return go(StoreF64{});
        case kStoreF32: return go(StoreF32{});
        case kStoreF16: return go(StoreF16{});
        case kStoreBF16: return go(StoreBF16{});
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
        if (host_table[i].tile_x != host_table[0].tile_x || host_table[i].vw != host_table[0].vw) return hipErrorInvalidValue;
        total += host_table[i].ntiles;
    }
    if (total != ntiles) return hipErrorInvalidValue;
    StepArgs a0 = host_table[0];
    a0.xcd_remap = xcd_remap;
    auto go = [&](auto St) -> hipError_t {
        using S = decltype(St);
        return with_width<S>(a0.vw, [&](auto Vc) {
            return launch_batch_v<S, decltype(Vc)::value>(odd, a0, dev_table, dev_tile_inst, ntiles, s);
        });
    };
    switch (store) {
        case kStoreF64: return go(StoreF64{});
        case kStoreF32: return go(StoreF32{});
        case kStoreF16: return go(StoreF16{});
        case kStoreBF16: return go(StoreBF16{});
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
template <typename S> struct CodecK { static constexpr auto fn = k_codec<S>; };

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

hipError_t launch_codec(int store, const float* in, float* out, long long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    // one thread per group; n threads cover the narrowest (one-element) groups
    return dispatch_store<CodecK>(store, blocks_for(n, 256), dim3(256), s, in, out, n);
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
