// Compile-time velocity sets D2Q37 and D3Q107 (Sec. IV, Tables I and II).
//
// Every group of a table is the set of all axis permutations and sign
// changes of one representative vector (in units of the scale r).  The
// library orders the velocities as: the rest velocity first, then opposite
// pairs (m, -m) next to each other, group by group.  Pairing lets the
// equilibrium evaluate the even and odd parts of its polynomial in c = xi.u
// once per pair.
#pragma once

#include <cstdint>

namespace lbm {

struct Vel {
    int x, y, z;   // lattice vector e_i (units of cells per step)
    int group;     // index of the table group (= shell |e|^2)
};

template <int D> struct VelSetTraits;
template <> struct VelSetTraits<2> { static constexpr int Q = 37, G = 8; };
template <> struct VelSetTraits<3> { static constexpr int Q = 107, G = 10; };

// Group representatives, in table order.
constexpr int kRep2[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {2, 0, 0},
                             {2, 1, 0}, {3, 0, 0}, {3, 1, 0}, {3, 3, 0}};
constexpr int kRep3[10][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {1, 1, 1},
                              {2, 0, 0}, {2, 1, 1}, {2, 2, 0}, {2, 2, 2},
                              {3, 0, 0}, {3, 1, 1}};

template <int D> struct VelSet {
    static constexpr int Q = VelSetTraits<D>::Q;
    static constexpr int G = VelSetTraits<D>::G;
    Vel v[Q];
    int rep[G][3];
    int qn[G];         // |e|^2 of each group
    int count[G];      // members per group
};

namespace detail {

constexpr bool same(const Vel& a, int x, int y, int z) {
    return a.x == x && a.y == y && a.z == z;
}

// "canonical" member of a +/- pair: first nonzero component positive
constexpr bool positive(int x, int y, int z) {
    return x > 0 || (x == 0 && (y > 0 || (y == 0 && z > 0)));
}

}  // namespace detail

template <int D> constexpr VelSet<D> make_velset() {
    VelSet<D> s{};
    int n = 0;
    constexpr int perms3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                  {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    constexpr int perms2[2][3] = {{0, 1, 2}, {1, 0, 2}};
    for (int g = 0; g < VelSet<D>::G; ++g) {
        int rep[3] = {0, 0, 0};
        for (int k = 0; k < 3; ++k) rep[k] = (D == 2 ? kRep2[g][k] : kRep3[g][k]);
        for (int k = 0; k < 3; ++k) s.rep[g][k] = rep[k];
        s.qn[g] = rep[0] * rep[0] + rep[1] * rep[1] + rep[2] * rep[2];
        const int first = n;
        if (g == 0) {
            s.v[n++] = Vel{0, 0, 0, 0};
            s.count[g] = 1;
            continue;
        }
        const int np = D == 2 ? 2 : 6;
        // members in a fixed order: sign patterns outer, permutations inner
        for (int sg = 0; sg < (1 << D); ++sg) {
            for (int p = 0; p < np; ++p) {
                int c[3] = {0, 0, 0};
                for (int k = 0; k < D; ++k) {
                    const int src = D == 2 ? perms2[p][k] : perms3[p][k];
                    const int sign = (sg >> k) & 1 ? -1 : 1;
                    c[k] = sign * rep[src];
                }
                if (!detail::positive(c[0], c[1], c[2])) continue;
                bool dup = false;
                for (int j = first; j < n; ++j)
                    if (detail::same(s.v[j], c[0], c[1], c[2])) dup = true;
                if (dup) continue;
                s.v[n++] = Vel{c[0], c[1], c[2], g};
                s.v[n++] = Vel{-c[0], -c[1], -c[2], g};
            }
        }
        s.count[g] = n - first;
    }
    return s;
}

template <int D> inline constexpr VelSet<D> kVelSet = make_velset<D>();

static_assert(kVelSet<2>.v[36].group == 7, "D2Q37 must have 37 velocities");
static_assert(kVelSet<3>.v[106].group == 9, "D3Q107 must have 107 velocities");
static_assert(kVelSet<2>.count[4] == 8 && kVelSet<2>.count[6] == 8,
              "Perm(2r,r) and Perm(3r,r) have 8 members each");
static_assert(kVelSet<3>.count[5] == 24 && kVelSet<3>.count[9] == 24,
              "Perm(2r,r,r) and Perm(3r,r,r) have 24 members each");

}  // namespace lbm
