// Velocity sets of the GPU path.  Standard D2Q9 and D3Q19 with c_s^2 = 1/3;
// directions are stored in +/- pairs (opp of q is q^1 for q > 0 after the
// rest velocity), so bounce-back partners are adjacent.
#pragma once

namespace eelbm {

struct D2Q9 {
    static constexpr int D = 2;
    static constexpr int Q = 9;
    static constexpr int NPI = 3;  // independent components of a symmetric 2x2 tensor
    static constexpr int c[9][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                                    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
    static constexpr int opp[9] = {0, 2, 1, 4, 3, 6, 5, 8, 7};
    static constexpr double w[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                                    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
};

struct D3Q19 {
    static constexpr int D = 3;
    static constexpr int Q = 19;
    static constexpr int NPI = 6;
    static constexpr int c[19][3] = {{0, 0, 0},   {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                                     {0, 0, 1},   {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                                     {-1, 1, 0},  {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                     {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    static constexpr double w[19] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                                     1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
};

// index of the (a, b) component of a symmetric tensor stored as
// xx, yy, [zz], xy, [xz, yz]
template <int D>
constexpr int sym(int a, int b) {
    if (a == b) return a;
    if (a > b) { int t = a; a = b; b = t; }
    return D == 2 ? 2 : (a == 0 ? (b == 1 ? 3 : 4) : 5);
}

}  // namespace eelbm
