// D3Q19 lattice constants for the device kernels.
//
// Velocity numbering follows Table A-1 of Han, Ooka & Kikumoto (arXiv
// 2009.04352): odd/even pairs are opposite (1/2, 3/4, ...), 13/14, 15/16 and
// 17/18 carry mixed signs.  Weights are those of the standard D3Q19 BGK model
// (Qian, d'Humieres & Lallemand 1992), which the paper cites for the scheme.
#pragma once

namespace lbmwf {

constexpr int kQ = 19;

constexpr int kEx[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0};
constexpr int kEy[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 1, -1};
constexpr int kEz[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 1, -1, 1};

// opposite direction: e_opp(a) = -e_a (pairs are adjacent in the numbering)
constexpr int opp(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }

// reflection in a wall normal to y: e = (ex, -ey, ez)
constexpr int mirror_y(int a)
{
    for (int b = 0; b < kQ; ++b)
        if (kEx[b] == kEx[a] && kEy[b] == -kEy[a] && kEz[b] == kEz[a]) return b;
    return -1;
}

constexpr int norm2(int a) { return kEx[a] * kEx[a] + kEy[a] * kEy[a] + kEz[a] * kEz[a]; }

template <typename R>
constexpr R weight(int a)
{
    return norm2(a) == 0 ? R(1) / R(3) : (norm2(a) == 1 ? R(1) / R(18) : R(1) / R(36));
}

// a population crosses the bottom wall (y < 0) when it moves in -y, the top
// wall when it moves in +y; the populations entering the fluid through a wall
// are the opposite ones.
constexpr bool enters_bottom(int a) { return kEy[a] == 1; }
constexpr bool enters_top(int a) { return kEy[a] == -1; }

// populations whose wall reflection is a mirror image (tangential part kept):
// every wall-crossing direction except the wall-normal ones.
constexpr bool is_tangential(int a) { return kEx[a] != 0 || kEz[a] != 0; }

// Wall nodes: the populations the bottom wall node sends into the fluid
// (e_y = +1), in the order of the wall-node rings; the top wall's are their
// mirror images.  in_index_b(a): position of a in that list (-1 if absent).
constexpr int kInB[5] = {3, 7, 11, 14, 17};
constexpr int in_index_b(int a)
{
    for (int k = 0; k < 5; ++k)
        if (kInB[k] == a) return k;
    return -1;
}
// ring element of the arrival a mirror reflection turns into kInB[k]
// (opp(mirror_y(kInB[k])) holds it; bounce-back uses element k itself)
constexpr int node_spec(int k) { return in_index_b(opp(mirror_y(kInB[k]))); }

static_assert(opp(7) == 8 && opp(13) == 14 && opp(17) == 18, "pair numbering");
static_assert(node_spec(0) == 0 && node_spec(1) == 3 && node_spec(2) == 4 && node_spec(3) == 1 && node_spec(4) == 2,
              "mirror pairs 7-13, 14-8, 11-18, 17-12 of Eq. 14");
static_assert(mirror_y(7) == 13 && mirror_y(14) == 8 && mirror_y(11) == 18 && mirror_y(17) == 12,
              "mirror pairs of the WFB collision");

}  // namespace lbmwf
