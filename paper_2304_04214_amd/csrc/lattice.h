// Device-side D3Q19 lattice of the library (Sec. II.A, Eq. (1)-(2)).
// Index order: lexicographic in (c_z, c_y, c_x); opposite(i) = 18 - i.
#pragma once

namespace lbm {

constexpr int Q = 19;
constexpr int CX[Q] = {0, -1, 0, 1, 0, -1, 0, 1, -1, 0, 1, -1, 0, 1, 0, -1, 0, 1, 0};
constexpr int CY[Q] = {-1, 0, 0, 0, 1, -1, -1, -1, 0, 0, 0, 1, 1, 1, -1, 0, 0, 0, 1};
constexpr int CZ[Q] = {-1, -1, -1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1};
constexpr double WD[Q] = {1.0 / 36, 1.0 / 36, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 18,
                          1.0 / 36, 1.0 / 18, 1.0 / 3,  1.0 / 18, 1.0 / 36, 1.0 / 18, 1.0 / 36,
                          1.0 / 36, 1.0 / 36, 1.0 / 18, 1.0 / 36, 1.0 / 36};
// Mirror image in y (specular reflection at a wall normal to y).
constexpr int REFLY[Q] = {4, 1, 2, 3, 0, 11, 12, 13, 8, 9, 10, 5, 6, 7, 18, 15, 16, 17, 14};
// Directions with c_x = -1 (outlet unknowns, outlet history order) and c_x = +1.
constexpr int OUT5[5] = {1, 5, 8, 11, 15};
constexpr int opp(int i) { return 18 - i; }

// Squared norms of the moment-basis rows, diag(M M^T) (Appendix A.1 basis).
constexpr double DNORM[Q] = {19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8};

}  // namespace lbm
