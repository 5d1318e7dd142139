// Orders p = 3, 4: hierarchic basis tables and the kernels that use them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace chom {
namespace hp {

// Compile-time shape of order P: element DOFs NE, dimension M of P_{P-1},
// padded operand shapes of the two element products (16-row tiles, 4-deep steps):
//   G = DA X with DA [MA][KA] = [D_1; D_2; D_3] (3M x NE, padded),
//   Y = DB H with DB [MB][KB] = DA^T (NE x 3M, padded).
template <int P> struct Shape;
template <> struct Shape<3> {
    static constexpr int NE = 20, M = 10, MA = 32, KA = 20, MB = 32, KB = 32;
};
template <> struct Shape<4> {
    static constexpr int NE = 35, M = 20, MA = 64, KA = 36, MB = 48, KB = 60;
};

// Host tables of one order (exact rationals evaluated in FP64).
struct HostTables {
    int p = 0, ne = 0, m = 0;
    std::vector<int> off;        // [6][ne][3]: lattice offset (units 1/p cell) of each local DOF per tet type
    std::vector<double> W;       // [ne]: (1/|e|) int phi_i
    std::vector<double> Wd;      // [3][ne]: (1/|e|) int d phi_i / d xi_k, k = 1..3
    std::vector<double> D;       // [3][m][ne]: derivative coefficients in a mass-orthonormal P_{p-1} basis
    std::vector<double> S;       // [9][ne][ne]: (1/|e|) int d_k phi_i d_l phi_j = D_k^T D_l
    std::vector<double> Sd;      // [9][ne]: diagonal of S
};

// Builds the tables of order p (3 or 4); false for other orders.
bool build_tables(int p, HostTables &t);

// Values of the order-p basis functions at barycentric point lam[4].
bool eval_basis(int p, const double lam[4], double *out);

}  // namespace hp
}  // namespace chom
