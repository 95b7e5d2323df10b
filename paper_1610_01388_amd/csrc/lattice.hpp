// lattice.hpp -- velocity sets of the GPU library (Sec. 4.1 names D2Q9,
// D3Q19 and D3Q27; the paper does not list them, these are the standard
// sets with the standard weights).
//
// Order: the rest velocity first, then opposite pairs (2k-1, 2k), so that
// opp(i) = i + 1 for odd i and i - 1 for even i > 0.  D3Q19 is the first 19
// entries of D3Q27 (faces, then edges), D3Q27 adds the 8 corners.
#pragma once

namespace lbm {

template <int LAT> struct Lattice;

template <> struct Lattice<0> {  // D2Q9
    static constexpr int D = 2, Q = 9;
    static constexpr int cx[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
    static constexpr int cy[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

#define LBM_D3_CX 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0
#define LBM_D3_CY 0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1
#define LBM_D3_CZ 0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1

template <> struct Lattice<1> {  // D3Q19
    static constexpr int D = 3, Q = 19;
    static constexpr int cx[19] = {LBM_D3_CX};
    static constexpr int cy[19] = {LBM_D3_CY};
    static constexpr int cz[19] = {LBM_D3_CZ};
    static constexpr double w[19] = {1.0 / 3,
                                     1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

template <> struct Lattice<2> {  // D3Q27
    static constexpr int D = 3, Q = 27;
    static constexpr int cx[27] = {LBM_D3_CX, 1, -1, 1, -1, 1, -1, -1, 1};
    static constexpr int cy[27] = {LBM_D3_CY, 1, -1, 1, -1, -1, 1, 1, -1};
    static constexpr int cz[27] = {LBM_D3_CZ, 1, -1, -1, 1, 1, -1, 1, -1};
    static constexpr double w[27] = {8.0 / 27,
                                     2.0 / 27, 2.0 / 27, 2.0 / 27, 2.0 / 27, 2.0 / 27, 2.0 / 27,
                                     1.0 / 54, 1.0 / 54, 1.0 / 54, 1.0 / 54, 1.0 / 54, 1.0 / 54,
                                     1.0 / 54, 1.0 / 54, 1.0 / 54, 1.0 / 54, 1.0 / 54, 1.0 / 54,
                                     1.0 / 216, 1.0 / 216, 1.0 / 216, 1.0 / 216,
                                     1.0 / 216, 1.0 / 216, 1.0 / 216, 1.0 / 216};
};

#undef LBM_D3_CX
#undef LBM_D3_CY
#undef LBM_D3_CZ

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

}  // namespace lbm
