// Momentum stencils of the HIP path, as compile-time tables.
//
// SPH26 (paper Sec. V "spherical D3Q27", Sec. III B off-lattice set): the 26
// non-zero directions of the 3x3x3 cube, normalised; weights of the 26-point
// Lebedev rule (faces 1/21, edges 4/105, corners 9/280), exact for angular
// averages of degree <= 7.  The zero momentum carries weight 0 and is not
// stored.  CIRC8: 8 in-plane unit directions at 2 pi q / 8, weight 1/8.
//
// Directions are stored grouped in "in-plane classes": members of a class
// share the weight and the in-plane projection (ux, uy) up to sign, and the
// out-of-plane |vz|.  Within a class the members moving along +u come first
// (nplus of them), then the antipodes moving along -u (nminus).  A class with
// u = 0 (the two z faces) has only plus members.  Every step quantity of a
// member -- the Anderson-Witting rate, the equilibrium, the force increment --
// depends on the direction only through beta.u, |vz| and the sign, so it is
// computed once per class and sign.
#pragma once

#include <cstdint>

namespace rlbm {

struct Dir {
    int cx, cy, cz;   // integer cube direction; v = c / |c|
};

struct DirClass {
    int first;        // index of the first member
    int nplus;        // members along +u
    int nminus;       // members along -u (antipodes, same order as the plus ones)
    int ncomp;        // non-zero cube components of the members (1, 2 or 3)
    int sx, sy;       // signs of (ux, uy) of the plus members
    double vz2;       // vz^2 of every member
    double w;         // quadrature weight of every member
};

constexpr double kInvSqrt2 = 0.70710678118654752440;
constexpr double kInvSqrt3 = 0.57735026918962576451;

constexpr double comp_mag(int ncomp) {
    return ncomp == 1 ? 1.0 : (ncomp == 2 ? kInvSqrt2 : kInvSqrt3);
}

struct Sph26 {
    static constexpr int Q = 26;
    static constexpr int NC = 9;
    static constexpr int D = 3;        // angular dimension: P = eps / 3
    static constexpr Dir dir[Q] = {
        {1, 0, 0},   {-1, 0, 0},                                    // class 0: x faces
        {0, 1, 0},   {0, -1, 0},                                    // class 1: y faces
        {0, 0, 1},   {0, 0, -1},                                    // class 2: z faces
        {1, 1, 0},   {-1, -1, 0},                                   // class 3: xy edges (+,+)
        {1, -1, 0},  {-1, 1, 0},                                    // class 4: xy edges (+,-)
        {1, 0, 1},   {1, 0, -1},  {-1, 0, -1},  {-1, 0, 1},         // class 5: xz edges
        {0, 1, 1},   {0, 1, -1},  {0, -1, -1},  {0, -1, 1},         // class 6: yz edges
        {1, 1, 1},   {1, 1, -1},  {-1, -1, -1}, {-1, -1, 1},        // class 7: corners (+,+)
        {1, -1, 1},  {1, -1, -1}, {-1, 1, -1},  {-1, 1, 1},         // class 8: corners (+,-)
    };
    static constexpr DirClass cls[NC] = {
        {0, 1, 1, 1, 1, 0, 0.0, 1.0 / 21.0},
        {2, 1, 1, 1, 0, 1, 0.0, 1.0 / 21.0},
        {4, 2, 0, 1, 0, 0, 1.0, 1.0 / 21.0},
        {6, 1, 1, 2, 1, 1, 0.0, 4.0 / 105.0},
        {8, 1, 1, 2, 1, -1, 0.0, 4.0 / 105.0},
        {10, 2, 2, 2, 1, 0, 0.5, 4.0 / 105.0},
        {14, 2, 2, 2, 0, 1, 0.5, 4.0 / 105.0},
        {18, 2, 2, 3, 1, 1, 1.0 / 3.0, 9.0 / 280.0},
        {22, 2, 2, 3, 1, -1, 1.0 / 3.0, 9.0 / 280.0},
    };
};

// z-mirror fold of Sph26.  Every state of the one-layer (N x N x 1) model is
// symmetric under v_z -> -v_z, so the two members of each mirror pair carry the
// same population; they are stored once, at the summed weight.  The members
// with v_z != 0 are represented by v_z > 0 (only |v_z| enters the step).
struct Sph17 {
    static constexpr int Q = 17;
    static constexpr int NC = 9;
    static constexpr int D = 3;        // angular dimension: P = eps / 3
    static constexpr Dir dir[Q] = {
        {1, 0, 0},  {-1, 0, 0},                                     // class 0: x faces
        {0, 1, 0},  {0, -1, 0},                                     // class 1: y faces
        {0, 0, 1},                                                  // class 2: z faces (pair)
        {1, 1, 0},  {-1, -1, 0},                                    // class 3
        {1, -1, 0}, {-1, 1, 0},                                     // class 4
        {1, 0, 1},  {-1, 0, 1},                                     // class 5: xz edges (pairs)
        {0, 1, 1},  {0, -1, 1},                                     // class 6: yz edges (pairs)
        {1, 1, 1},  {-1, -1, 1},                                    // class 7: corners (pairs)
        {1, -1, 1}, {-1, 1, 1},                                     // class 8: corners (pairs)
    };
    static constexpr DirClass cls[NC] = {
        {0, 1, 1, 1, 1, 0, 0.0, 1.0 / 21.0},
        {2, 1, 1, 1, 0, 1, 0.0, 1.0 / 21.0},
        {4, 1, 0, 1, 0, 0, 1.0, 2.0 / 21.0},
        {5, 1, 1, 2, 1, 1, 0.0, 4.0 / 105.0},
        {7, 1, 1, 2, 1, -1, 0.0, 4.0 / 105.0},
        {9, 1, 1, 2, 1, 0, 0.5, 8.0 / 105.0},
        {11, 1, 1, 2, 0, 1, 0.5, 8.0 / 105.0},
        {13, 1, 1, 3, 1, 1, 1.0 / 3.0, 9.0 / 140.0},
        {15, 1, 1, 3, 1, -1, 1.0 / 3.0, 9.0 / 140.0},
    };
};

struct Circ8 {
    static constexpr int Q = 8;
    static constexpr int NC = 4;
    static constexpr int D = 2;        // angular dimension: P = eps / 2
    static constexpr Dir dir[Q] = {
        {1, 0, 0},  {-1, 0, 0},
        {0, 1, 0},  {0, -1, 0},
        {1, 1, 0},  {-1, -1, 0},
        {1, -1, 0}, {-1, 1, 0},
    };
    static constexpr DirClass cls[NC] = {
        {0, 1, 1, 1, 1, 0, 0.0, 0.125},
        {2, 1, 1, 1, 0, 1, 0.0, 0.125},
        {4, 1, 1, 2, 1, 1, 0.0, 0.125},
        {6, 1, 1, 2, 1, -1, 0.0, 0.125},
    };
};

// Unit vector component of a direction (host and device).
constexpr double dir_comp(const Dir& d, int axis) {
    const int n = (d.cx != 0) + (d.cy != 0) + (d.cz != 0);
    const int c = axis == 0 ? d.cx : (axis == 1 ? d.cy : d.cz);
    return c * comp_mag(n);
}

// Index of the z mirror (cx, cy, -cz) of direction q of the 26-direction set.
constexpr int mirror_of(int q) {
    for (int p = 0; p < Sph26::Q; ++p)
        if (Sph26::dir[p].cx == Sph26::dir[q].cx && Sph26::dir[p].cy == Sph26::dir[q].cy &&
            Sph26::dir[p].cz == -Sph26::dir[q].cz)
            return p;
    return -1;
}

}  // namespace rlbm
