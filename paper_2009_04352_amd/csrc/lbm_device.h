// Device building blocks of the fused step: lattice loops, the FP64 wall
// function, the collision, wave reductions and the store-format lane groups.
// Included by every translation unit that instantiates step kernels.
//
// Method: Han, Ooka & Kikumoto, "A wall function approach in lattice
// Boltzmann method" (arXiv 2009.04352).
#pragma once
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

// Tile of a block.  Blocks are dispatched round-robin over the 8 XCDs (block
// b to XCD b mod 8).  remap = 0 keeps tile = b.  remap = c + 1 hands the XCDs
// chunks of 2^c consecutive tiles in turn: XCD k works through chunks k,
// k + 8, k + 16, ..., so each XCD's L2 sees runs of neighbouring tiles and
// every XCD gets an even share of each region of the grid (the wall rows'
// extra work included).  Tiles past the last whole round of 8 chunks keep
// tile = b.
__device__ __forceinline__ int tile_of_block(int b, int ntiles, int remap)
{
    if (remap <= 0) return b;
    const int c = remap - 1;
    const int full = (ntiles >> (c + 3)) << (c + 3);
    if (b >= full) return b;
    const int k = b & 7, j = b >> 3;
    return ((((j >> c) << 3) + k) << c) + (j & ((1 << c) - 1));
}

// Tile at launch position u when the bricks are spread over the launch (see
// set_spread on the host): position u is tile i of chunk G = u >> spread;
// round q = G / nbricks of chunks takes chunk q of brick (G + q) mod nbricks
// (rotated) or G mod nbricks.  A bijection on the tiles; identity when
// spread < 0.
__device__ __forceinline__ int spread_tile(int u, const StepArgs& p)
{
    if (p.spread < 0) return u;
    const int G = u >> p.spread, i = u & ((1 << p.spread) - 1);
    const int q = fdiv(G, p.fd_nbricks);
    int g = G - q * p.nbricks;
    if (p.spread_rot) {
        g += q - fdiv(q, p.fd_nbricks) * p.nbricks;   // (G + q) mod nbricks
        if (g >= p.nbricks) g -= p.nbricks;
    }
    return g * p.tiles_per_brick + (q << p.spread) + i;
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

// Friction velocities from Spalding's law (Eq. 16-17) for NC wall cells at
// once.  In p = u+ = U / u_tau with R = y1 U / nu the law reads
// H(p) = p Sp(p) - R = 0.  H is increasing and convex for p > 0, so Newton's
// method converges from any positive start (after at most one step it is
// right of the root and then decreases monotonically); it stops when
// |p_{k+1} - p_k| <= tol p_{k+1}.
//
// The FP64 iteration starts from an FP32 estimate: the log law
// u+ = ln(y+) / kappa + B with y+ = R / p, iterated as a fixed point (it
// contracts for p > 1 / kappa), taken when it is below the viscous guess
// sqrt(R); then FP32 Newton steps on H until the change is below 1e-6, with
// the hardware reciprocal in place of divisions.  Only the start of the
// FP64 iteration depends on it, and through it only the iteration count.
//
// The NC solves run side by side (independent dependency chains); each cell
// keeps its own stopping step, so every cell gets the value a solve of its
// own would give.  Cells with U = 0 get u_tau = 0.
// `iters` is the largest FP64 step count of the live cells, `fail` is set if
// any live cell reached maxit without meeting the stop.
template <int NC>
__device__ __forceinline__ void wall_utau_n(const double (&U)[NC], double y1, double nu, double kappa, double bconst,
                                            double ekb, double tol, int maxit, double (&ut)[NC], int& iters,
                                            bool& fail)
{
    double R[NC], p[NC];
    bool live[NC], run[NC];
    int cnt[NC];
    const float kf = (float)kappa, ekf = (float)ekb, ikf = 1.0f / kf;
    float pf[NC], Rf[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        live[c] = U[c] > 0.0;
        R[c] = live[c] ? y1 * U[c] / nu : 1.0;
        Rf[c] = (float)R[c];
        pf[c] = sqrtf(Rf[c]);
        float pl = pf[c];
#pragma unroll
        for (int i = 0; i < 3; ++i) pl = fmaf(__logf(Rf[c] * __builtin_amdgcn_rcpf(pl)), ikf, (float)bconst);
        if (pl > 1.0f && pl < pf[c]) pf[c] = pl;
        run[c] = true;
    }
    for (int i = 0; i < 6; ++i) {
        bool any = false;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const float q = pf[c];
            const float k = kf * q, ek = __expf(k), k2 = 0.5f * k * k;
            const float br = ek - 1.0f - k - k2;
            const float sp = q + ekf * (br - k2 * k * (1.0f / 3.0f));
            const float dsp = 1.0f + kf * ekf * br;
            const float pn = q - (q * sp - Rf[c]) * __builtin_amdgcn_rcpf(sp + q * dsp);
            if (run[c]) {
                if (!(pn > 0.0f) || !(pn < INFINITY)) {
                    run[c] = false;
                } else {
                    run[c] = !(fabsf(pn - q) <= 1e-6f * pn);
                    pf[c] = pn;
                }
            }
            any = any || run[c];
        }
        if (!any) break;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        p[c] = (pf[c] > 0.0f && pf[c] < INFINITY) ? (double)pf[c] : sqrt(R[c]);
        run[c] = live[c];
        cnt[c] = 0;
    }
    for (int it = 1; it <= maxit; ++it) {
        bool any = false;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double q = p[c];
            const double k = kappa * q;
            const double ek = exp(k);
            const double k2 = 0.5 * k * k;
            const double br = ek - 1.0 - k - k2;              // e^k - 1 - k - k^2/2
            const double sp = q + ekb * (br - k2 * k * (1.0 / 3.0));
            const double dsp = 1.0 + kappa * ekb * br;
            const double pn = q - (q * sp - R[c]) / (sp + q * dsp);
            if (run[c]) {
                cnt[c] = it;
                run[c] = !(fabs(pn - q) <= tol * pn);
                p[c] = pn;
            }
            any = any || run[c];
        }
        if (!any) break;
    }
    iters = 0;
    fail = false;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        iters = max(iters, cnt[c]);
        fail = fail || run[c];
        ut[c] = live[c] ? U[c] / p[c] : 0.0;
    }
}

// One cell (U > 0) of the above: the device Newton probe uses it.
__device__ __forceinline__ double wall_utau(double U, double y1, double nu, double kappa, double bconst, double ekb,
                                            double tol, int maxit, int& iters, bool& fail)
{
    const double u[1] = {U};
    double ut[1];
    wall_utau_n<1>(u, y1, nu, kappa, bconst, ekb, tol, maxit, ut, iters, fail);
    return ut[0];
}

struct WallRecord {
    double taux, tauz, utau, U;
};

// Density and wall-parallel velocity of the gathered (free-slip) populations
// of a wall cell, with the half-force shift; returns |v_par| in FP64.
template <typename R>
__device__ __forceinline__ double wall_velocity(const R (&f)[kQ], R fx, R& rho, R& vx, R& vz)
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
    rho = R(1) + drho;
    vx = (jx + R(0.5) * fx) / rho;
    vz = jz / rho;
    const double dx = (double)vx, dz = (double)vz;
    return sqrt(dx * dx + dz * dz);
}

// Wall stress from the friction velocity: tau_w = rho u_tau^2 split against
// the wall-parallel velocity (Eq. 15, 17); zero when U = 0.
__device__ __forceinline__ WallRecord wall_record(double rho, double vx, double vz, double U, double ut)
{
    WallRecord rec{0.0, 0.0, 0.0, U};
    if (U > 0.0) {
        const double tauw = rho * ut * ut;
        rec.taux = -(vx / U) * tauw;
        rec.tauz = -(vz / U) * tauw;
        rec.utau = ut;
    }
    return rec;
}

// The bounce correction: +-tau/2 on the four reflected diagonal populations
// (Eq. 13-14 with dt = dy = 1), hx = tau_x / 2 and hz = tau_z / 2.  Top wall:
// the bottom rule mirrored in y.
template <typename R>
__device__ __forceinline__ void wfb_apply(R (&f)[kQ], bool top, R hx, R hz)
{
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
}

// WFB correction of the gathered (free-slip) populations of one wall cell:
// tau_w from the wall function, split along the wall-parallel velocity and
// applied as the bounce correction.
template <typename R>
__device__ __forceinline__ WallRecord wfb_correct(R (&f)[kQ], bool top, double fx, double y1, double nu0,
                                                  double kappa, double bconst, double ekb, double tol, int maxit,
                                                  int& iters, bool& fail)
{
    R rho, vx, vz;
    const double U[1] = {wall_velocity<R>(f, (R)fx, rho, vx, vz)};
    double ut[1];
    wall_utau_n<1>(U, y1, nu0, kappa, bconst, ekb, tol, maxit, ut, iters, fail);
    const WallRecord rec = wall_record((double)rho, (double)vx, (double)vz, U[0], ut[0]);
    wfb_apply<R>(f, top, (R)(0.5 * rec.taux), (R)(0.5 * rec.tauz));
    return rec;
}

// ---------------------------------------------- MRT basis (Sec. 3.1, [40])

// Moment m_k of velocity a in the D3Q19 basis of d'Humieres et al. (2002):
// polynomials of e that are orthogonal over the 19 velocities.  Rows 0, 3,
// 5, 7 are density and momentum; 9, 11, 13-15 the viscous stresses; the
// others (energy 1, energy square 2, heat flux 4, 6, 8, fourth-order
// normal stresses 10, 12, third-order 16-18) are not hydrodynamic and relax
// at rates of their own.
constexpr int mrt_row(int k, int a)
{
    const int ex = kEx[a], ey = kEy[a], ez = kEz[a], e2 = ex * ex + ey * ey + ez * ez;
    switch (k) {
        case 0: return 1;
        case 1: return 19 * e2 - 30;
        case 2: return (21 * e2 * e2 - 53 * e2 + 24) / 2;   // 12, -4, 1 for |e|^2 = 0, 1, 2
        case 3: return ex;
        case 4: return (5 * e2 - 9) * ex;
        case 5: return ey;
        case 6: return (5 * e2 - 9) * ey;
        case 7: return ez;
        case 8: return (5 * e2 - 9) * ez;
        case 9: return 3 * ex * ex - e2;
        case 10: return (3 * e2 - 5) * (3 * ex * ex - e2);
        case 11: return ey * ey - ez * ez;
        case 12: return (3 * e2 - 5) * (ey * ey - ez * ez);
        case 13: return ex * ey;
        case 14: return ey * ez;
        case 15: return ex * ez;
        case 16: return (ey * ey - ez * ez) * ex;
        case 17: return (ez * ez - ex * ex) * ey;
        default: return (ex * ex - ey * ey) * ez;
    }
}

constexpr int mrt_norm(int k)
{
    int n = 0;
    for (int a = 0; a < kQ; ++a) n += mrt_row(k, a) * mrt_row(k, a);
    return n;
}

static_assert(mrt_norm(1) == 2394 && mrt_norm(2) == 252 && mrt_norm(10) == 72 && mrt_norm(16) == 8, "basis norms");
// entries the reduced moments of the collision below rely on
static_assert(mrt_row(1, 0) == -30 && mrt_row(1, 1) == -11 && mrt_row(1, 7) == 8 && mrt_row(2, 0) == 12 &&
              mrt_row(2, 1) == -4 && mrt_row(2, 7) == 1, "energy rows");
static_assert(mrt_row(4, 1) == -4 && mrt_row(4, 7) == 1 && mrt_row(10, 1) == -4 && mrt_row(10, 3) == 2 &&
              mrt_row(10, 7) == mrt_row(9, 7) && mrt_row(10, 11) == mrt_row(9, 11) && mrt_row(12, 3) == -2 &&
              mrt_row(12, 5) == 2 && mrt_row(12, 7) == mrt_row(11, 7) && mrt_row(12, 9) == mrt_row(11, 9),
              "heat-flux and fourth-order rows");

// The non-hydrodynamic moments and the rate (index into MrtRates::s) each
// relaxes at: energy, energy square, heat flux, fourth-order normal
// stresses, third-order moments.
constexpr int kMrtNH[10] = {1, 2, 4, 6, 8, 10, 12, 16, 17, 18};
constexpr int kMrtRate[10] = {0, 1, 2, 2, 2, 3, 3, 4, 4, 4};

template <typename R>
struct MrtRates {
    R s[5];   // energy, energy square, heat flux, fourth-order normal stress, third-order
};

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
// 3 e_x (per unit force along x); both halves of the update are then
// polynomials in e.u whose coefficients depend only on the weight class.
//
// MRT (the paper's collision, [40]): the BGK result plus, for each
// non-hydrodynamic moment k, M^-1 of (omega - s_k) (n_k + F_k / 2), where
// n = M (f - f_eq) and F = M (force term): the difference between relaxing
// that moment at s_k (with the force added as (I - S/2) M F) and at omega.
// The stress moments relax at omega = 1/tau_e in both, density and
// momentum are conserved (their rates do not enter).
template <typename R, bool MRT = false>
__device__ __forceinline__ Moments<R> collide(R (&f)[kQ], R tau0, R cs2_18, R fx, const MrtRates<R>* mr = nullptr)
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
    const R t0 = fmad(rho, -usq, drho);          // drho - rho * 1.5 u.u

    // MRT: x_k = n_k + F_k / 2 of the non-hydrodynamic moments, i.e. the
    // moments of g = f - f_eq + F / 2.  g carries no mass and no momentum, and
    // its second moments are the non-equilibrium stress plus half of
    // u F + F u (for F along x: u_x F_x on the xx entry, which enters below,
    // and off-diagonal terms, which do not).  With
    //   T = tr = p_xx + p_yy + p_zz + u_x F_x,
    //   P9 = 3 (xx) - tr = 2 p_xx - p_yy - p_zz + 2 u_x F_x,  P11 = (yy) - (zz) = p_yy - p_zz,
    // the sums gs and differences gd of g over the axis pairs 1, 3, 5 and
    // the differences over the diagonal pairs, the rows reduce to
    //   x1 = 19 T,  x2 = -(5.5 T + 10.5 (gs1 + gs3 + gs5)),
    //   x4 = -5 gd1,  x6 = -5 gd3,  x8 = -5 gd5,
    //   x10 = P9 - 6 gs1 + 3 (gs3 + gs5),  x12 = P11 + 3 (gs5 - gs3),
    // and the third-order rows 16-18, which live on the diagonal pairs only.
    // Per pair (a, opp a) of the weight class w,
    //   gs = s - w (2 t0 + 9 rho (e.u)^2 + 3 u_x Fx - 9 e_x (e.u) Fx),
    //   gd = d - 3 w (2 rho e.u - e_x Fx).
    R xk[10] = {};
    if constexpr (MRT) {
        R gs[kQ], gd[kQ];   // indexed like s and d
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            if constexpr (a % 2 == 1) {
                constexpr R w = weight<R>(a);
                R eu = R(0);
                if constexpr (kEx[a] == 1) eu = ux;
                if constexpr (kEy[a] == 1) eu = (kEx[a] != 0) ? eu + uy : uy;
                if constexpr (kEy[a] == -1) eu = eu - uy;
                if constexpr (kEz[a] == 1) eu = (kEx[a] != 0 || kEy[a] != 0) ? eu + uz : uz;
                if constexpr (kEz[a] == -1) eu = eu - uz;
                const R ex_fx = (kEx[a] != 0) ? fx : R(0);
                if constexpr (a <= 5)
                    gs[a] = s[a] - w * fmad(R(9) * rho * eu, eu, fmad(R(3) * ux, fx, fmad(R(-9) * eu, ex_fx, R(2) * t0)));
                gd[a] = d[a] - (R(3) * w) * fmad(R(2) * rho, eu, -ex_fx);
            }
        });
        const R uxfx = ux * fx;
        const R tr = ((pxx + pyy) + pzz) + uxfx;
        const R p9 = fmad(R(2), pxx + uxfx, -(pyy + pzz));
        const R p11 = pyy - pzz;
        const R ax = (gs[1] + gs[3]) + gs[5];
        xk[0] = R(19) * tr;
        xk[1] = -fmad(R(5.5), tr, R(10.5) * ax);
        xk[2] = R(-5) * gd[1];
        xk[3] = R(-5) * gd[3];
        xk[4] = R(-5) * gd[5];
        xk[5] = fmad(R(-6), gs[1], fmad(R(3), gs[3] + gs[5], p9));
        xk[6] = fmad(R(3), gs[5] - gs[3], p11);
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            if constexpr (a % 2 == 1 && a >= 7) {
#pragma unroll
                for (int i = 7; i < 10; ++i) {
                    const int c = mrt_row(kMrtNH[i], a);
                    if (c != 0) xk[i] = fmad(R(c), gd[a], xk[i]);
                }
            }
        });
    }

    {   // rest population: e = 0
        constexpr R w = weight<R>(0);
        const R heq = w * t0;
        f[0] = fmad(-om, f[0] - heq, f[0]) + (w * fc) * m3ux;
    }
    // Per weight class (c = 0: 1/18, 1: 1/36) the pair update is linear in
    // e.u and (e.u)^2:
    //   S = omh s + A (e.u)^2 + C e_x e.u + B,   D = omh d + E e.u + G e_x
    // with A = 4.5 om w rho, E = 3 om w rho, B = om w t0 - 3 w fc ux,
    // C = 9 w fc, G = 3 w fc (the odd member of every pair has e_x = 0 or 1).
    const R rho45 = R(4.5) * rho, rho3 = R(3) * rho;
    R cA[2], cB[2], cC[2], cE[2], cG[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const R w = c == 0 ? weight<R>(1) : weight<R>(7);
        const R omw = om * w, fcw = w * fc;
        cA[c] = rho45 * omw;
        cE[c] = rho3 * omw;
        cB[c] = fmad(omw, t0, m3ux * fcw);
        cC[c] = R(9) * fcw;
        cG[c] = R(3) * fcw;
    }
    for_each_dir([&](auto A) {
        constexpr int a = decltype(A)::value;
        if constexpr (a % 2 == 1) {
            constexpr int ex = kEx[a];
            static_assert(ex == 0 || ex == 1, "odd members move in +x or not at all");
            constexpr int c = norm2(a) == 1 ? 0 : 1;
            R eu = R(0);
            if constexpr (kEx[a] == 1) eu = ux;
            if constexpr (kEy[a] == 1) eu = (kEx[a] != 0) ? eu + uy : uy;
            if constexpr (kEy[a] == -1) eu = eu - uy;
            if constexpr (kEz[a] == 1) eu = (kEx[a] != 0 || kEy[a] != 0) ? eu + uz : uz;
            if constexpr (kEz[a] == -1) eu = eu - uz;
            // half sum and half difference of the post-collision pair
            const R sc = (ex != 0) ? fmad(cC[c], eu, cB[c]) : cB[c];
            const R S = fmad(omh, s[a], fmad(cA[c], eu * eu, sc));
            const R D = fmad(omh, d[a], (ex != 0) ? fmad(cE[c], eu, cG[c]) : cE[c] * eu);
            f[a] = S + D;
            f[a + 1] = S - D;
        }
    });
    if constexpr (MRT) {
        // c_k = (omega - s_k) x_k / |row k|^2, added back through M^T
        R ck[10];
#pragma unroll
        for (int i = 0; i < 10; ++i)
            ck[i] = (om - mr->s[kMrtRate[i]]) * xk[i] * R(1.0 / (double)mrt_norm(kMrtNH[i]));
        for_each_dir([&](auto A) {
            constexpr int a = decltype(A)::value;
            if constexpr (a == 0) {
                R v = R(0);
#pragma unroll
                for (int i = 0; i < 10; ++i)
                    if (mrt_row(kMrtNH[i], 0) != 0) v = fmad(R(mrt_row(kMrtNH[i], 0)), ck[i], v);
                f[0] += v;
            } else if constexpr (a % 2 == 1) {
                R ev = R(0), od = R(0);
#pragma unroll
                for (int i = 0; i < 10; ++i) {
                    const int k = kMrtNH[i];
                    const int c = mrt_row(k, a);
                    const bool even = (k == 1 || k == 2 || k == 10 || k == 12);
                    if (c != 0) {
                        if (even) ev = fmad(R(c), ck[i], ev);
                        else od = fmad(R(c), ck[i], od);
                    }
                }
                f[a] += ev + od;
                f[a + 1] += ev - od;
            }
        });
    }
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
    // element j of a group of 2- or 4-byte elements (V >= 2), as raw bits
    __device__ __forceinline__ static unsigned int elem(u32x2 v, int j)
    {
        static_assert(V >= 2 && kBytes <= 4, "groups of several elements");
        if constexpr (kBytes == 4) {
            return j == 0 ? v.x : v.y;
        } else {
            const unsigned int word = (j < 2) ? v.x : v.y;
            return (j & 1) ? (word >> 16) : (word & 0xffffu);
        }
    }
    // the group of V raw elements
    __device__ __forceinline__ static u32x2 from_elems(const unsigned int (&e)[V])
    {
        static_assert(V >= 2 && kBytes <= 4, "groups of several elements");
        if constexpr (kBytes == 4) return u32x2{e[0], e[1]};
        else if constexpr (V == 2) return u32x2{e[0] | (e[1] << 16), 0u};
        else return u32x2{e[0] | (e[1] << 16), e[2] | (e[3] << 16)};
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
    // elements k and k + 1 (k even) of a group of 2-byte elements, both
    // rounded to nearest even by one packed conversion
    __device__ __forceinline__ static void set_pair(u32x2& v, int k, float r0, float r1)
    {
        static_assert(kBytes == 2, "pairs of 2-byte elements");
        typedef float f32x2 __attribute__((ext_vector_type(2)));
        unsigned int word;
        if constexpr (S::kind == kStoreBF16) {
            typedef __bf16 b16x2 __attribute__((ext_vector_type(2)));
            word = __builtin_bit_cast(unsigned int, __builtin_convertvector((f32x2{r0, r1}), b16x2));
        } else {
            typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));
            word = __builtin_bit_cast(unsigned int, __builtin_convertvector((f32x2{r0, r1}), h16x2));
        }
        if (k < 2) v.x = word;
        else v.y = word;
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

}  // namespace lbmwf
