// Hierarchic basis of order p = 3, 4 on a tetrahedron and its exact tables.
//
// The paper uses hierarchic (Ainsworth-Coyle type) functions without printing
// them (Sec. 1, Sec. 7); any conforming hierarchic family spans the same space.
// The family here, in barycentric coordinates lam_0..lam_3 with the local vertex
// order equal to the global one (true for every Kuhn tet), is
//   vertex a:            lam_a
//   edge (a < b), k < p-1:  lam_a lam_b L_k(lam_b - lam_a)
//   face (a < b < c), i + j <= p-3:  lam_a lam_b lam_c L_i(lam_b - lam_a) L_j(2 lam_c - 1)
//   interior (p = 4):    lam_0 lam_1 lam_2 lam_3
// with L_k the Legendre polynomials.  A function's trace on an edge or face
// depends only on that entity's vertices in global order, so the space is
// conforming across tets and across periodic faces.
//
// Integrals are exact: (1/|e|) int lam^alpha = 6 alpha! / (|alpha| + 3)!.  The
// derivatives d/dxi_k = d/dlam_k - d/dlam_0 (xi_k = lam_k, k = 1..3) are
// polynomials of degree p-1; writing them in a basis of P_{p-1} that is
// orthonormal for the element mass product gives matrices D_k with
// (1/|e|) int d_k phi_i d_l phi_j = (D_k^T D_l)_ij, the factorisation the order-p
// operator applies on the matrix cores.
//
// Each local DOF is also given a point of the (p n + 1)^3 lattice: vertices at
// p x their grid point, edge DOF k at the (k+1)-th interior point of the edge,
// face DOF (i, j) at v_a + ((i+1)(v_b - v_a) + (j+1)(v_c - v_a)) / p, the
// interior DOF at the centroid; these points are distinct and cover the lattice,
// so the lattice index numbers the DOFs.
#include <array>
#include <cmath>
#include <map>
#include <vector>

#include "hp.h"

namespace chom {
namespace hp {
namespace {

using Mono = std::array<int, 4>;
using Poly = std::map<Mono, double>;

Poly var(int a) {
    Mono m{0, 0, 0, 0};
    m[a] = 1;
    return Poly{{m, 1.0}};
}
Poly constant(double c) { return Poly{{Mono{0, 0, 0, 0}, c}}; }

Poly add(const Poly &a, const Poly &b, double sb = 1.0) {
    Poly r = a;
    for (const auto &kv : b) r[kv.first] += sb * kv.second;
    return r;
}

Poly mul(const Poly &a, const Poly &b) {
    Poly r;
    for (const auto &x : a)
        for (const auto &y : b) {
            Mono m;
            for (int i = 0; i < 4; ++i) m[i] = x.first[i] + y.first[i];
            r[m] += x.second * y.second;
        }
    return r;
}

Poly dlam(const Poly &p, int a) {
    Poly r;
    for (const auto &kv : p) {
        if (kv.first[a] == 0) continue;
        Mono m = kv.first;
        const double c = kv.second * m[a];
        m[a] -= 1;
        r[m] += c;
    }
    return r;
}

Poly dxi(const Poly &p, int k) { return add(dlam(p, k), dlam(p, 0), -1.0); }

double fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

// (1/|e|) int over the tet
double integ(const Poly &p) {
    double s = 0.0;
    for (const auto &kv : p) {
        const Mono &m = kv.first;
        s += kv.second * 6.0 * fact(m[0]) * fact(m[1]) * fact(m[2]) * fact(m[3]) /
             fact(m[0] + m[1] + m[2] + m[3] + 3);
    }
    return s;
}

Poly legendre(int k, const Poly &x) {
    if (k == 0) return constant(1.0);
    if (k == 1) return x;
    // L_2 = (3 x^2 - 1) / 2
    return add(mul(constant(1.5), mul(x, x)), constant(-0.5));
}

double eval(const Poly &p, const double lam[4]) {
    double s = 0.0;
    for (const auto &kv : p) {
        double t = kv.second;
        for (int i = 0; i < 4; ++i)
            for (int e = 0; e < kv.first[i]; ++e) t *= lam[i];
        s += t;
    }
    return s;
}

// Substitute lam_0 = 1 - lam_1 - lam_2 - lam_3 (result has no lam_0).
Poly eliminate_lam0(const Poly &p) {
    const Poly one_minus = add(add(add(constant(1.0), var(1), -1.0), var(2), -1.0), var(3), -1.0);
    Poly r;
    for (const auto &kv : p) {
        Mono rest = kv.first;
        const int e0 = rest[0];
        rest[0] = 0;
        Poly term{{rest, kv.second}};
        for (int e = 0; e < e0; ++e) term = mul(term, one_minus);
        r = add(r, term);
    }
    return r;
}

struct Basis {
    int p;
    std::vector<Poly> f;                 // functions in local DOF order
    std::vector<std::array<int, 5>> ent; // kind (0 vertex, 1 edge, 2 face, 3 interior), verts a, b, c, sub-index
};

const int kEdge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
const int kFace[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};   // face f omits vertex f

Basis make_basis(int p) {
    Basis B;
    B.p = p;
    for (int a = 0; a < 4; ++a) {
        B.f.push_back(var(a));
        B.ent.push_back({0, a, -1, -1, 0});
    }
    for (int e = 0; e < 6; ++e) {
        const int a = kEdge[e][0], b = kEdge[e][1];
        const Poly ab = mul(var(a), var(b));
        const Poly x = add(var(b), var(a), -1.0);
        for (int k = 0; k <= p - 2; ++k) {
            B.f.push_back(mul(ab, legendre(k, x)));
            B.ent.push_back({1, a, b, -1, k});
        }
    }
    if (p >= 3)
        for (int fc = 0; fc < 4; ++fc) {
            const int a = kFace[fc][0], b = kFace[fc][1], c = kFace[fc][2];
            const Poly abc = mul(mul(var(a), var(b)), var(c));
            const Poly x = add(var(b), var(a), -1.0);
            const Poly y = add(mul(constant(2.0), var(c)), constant(-1.0));
            int sub = 0;
            for (int s = 0; s <= p - 3; ++s)
                for (int i = s; i >= 0; --i) {
                    const int j = s - i;
                    B.f.push_back(mul(abc, mul(legendre(i, x), legendre(j, y))));
                    B.ent.push_back({2, a, b, c, (i << 8) | j});
                    ++sub;
                }
        }
    if (p >= 4) {
        B.f.push_back(mul(mul(var(0), var(1)), mul(var(2), var(3))));
        B.ent.push_back({3, -1, -1, -1, 0});
    }
    return B;
}

}  // namespace

bool eval_basis(int p, const double lam[4], double *out) {
    if (p < 3 || p > 4) return false;
    const Basis B = make_basis(p);
    for (size_t i = 0; i < B.f.size(); ++i) out[i] = eval(B.f[i], lam);
    return true;
}

bool build_tables(int p, HostTables &t) {
    if (p < 3 || p > 4) return false;
    const Basis B = make_basis(p);
    const int ne = (int)B.f.size();
    t.p = p;
    t.ne = ne;
    // monomials xi^e of P_{p-1}
    std::vector<Mono> mono;
    for (int d = 0; d <= p - 1; ++d)
        for (int e1 = d; e1 >= 0; --e1)
            for (int e2 = d - e1; e2 >= 0; --e2) mono.push_back(Mono{0, e1, e2, d - e1 - e2});
    const int m = (int)mono.size();
    t.m = m;
    std::map<Mono, int> mono_idx;
    for (int a = 0; a < m; ++a) mono_idx[mono[a]] = a;
    // mass matrix of the monomials and its Cholesky factor M = R R^T
    std::vector<double> M(m * m), R(m * m, 0.0);
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            Mono s;
            for (int i = 0; i < 4; ++i) s[i] = mono[a][i] + mono[b][i];
            M[a * m + b] = integ(Poly{{s, 1.0}});
        }
    for (int j = 0; j < m; ++j) {
        double d = M[j * m + j];
        for (int k = 0; k < j; ++k) d -= R[j * m + k] * R[j * m + k];
        if (!(d > 0.0)) return false;
        R[j * m + j] = std::sqrt(d);
        for (int i = j + 1; i < m; ++i) {
            double s = M[i * m + j];
            for (int k = 0; k < j; ++k) s -= R[i * m + k] * R[j * m + k];
            R[i * m + j] = s / R[j * m + j];
        }
    }
    // derivative coefficients C^k [m][ne] and D_k = R^T C^k
    t.D.assign(3 * m * ne, 0.0);
    t.W.assign(ne, 0.0);
    t.Wd.assign(3 * ne, 0.0);
    for (int i = 0; i < ne; ++i) {
        t.W[i] = integ(B.f[i]);
        for (int k = 0; k < 3; ++k) {
            const Poly dk = dxi(B.f[i], k + 1);
            t.Wd[k * ne + i] = integ(dk);
            const Poly q = eliminate_lam0(dk);
            std::vector<double> c(m, 0.0);
            for (const auto &kv : q) {
                if (kv.second == 0.0) continue;
                const auto it = mono_idx.find(kv.first);
                if (it == mono_idx.end()) return false;   // degree above p-1: cannot happen
                c[it->second] += kv.second;
            }
            for (int a = 0; a < m; ++a) {
                double s = 0.0;
                for (int b = a; b < m; ++b) s += R[b * m + a] * c[b];   // (R^T c)_a
                t.D[(k * m + a) * ne + i] = s;
            }
        }
    }
    t.S.assign(9 * ne * ne, 0.0);
    t.Sd.assign(9 * ne, 0.0);
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l)
            for (int i = 0; i < ne; ++i)
                for (int j = 0; j < ne; ++j) {
                    double s = 0.0;
                    for (int a = 0; a < m; ++a) s += t.D[(k * m + a) * ne + i] * t.D[(l * m + a) * ne + j];
                    t.S[((k * 3 + l) * ne + i) * ne + j] = s;
                    if (i == j) t.Sd[(k * 3 + l) * ne + i] = s;
                }
    // lattice offsets per Kuhn tet type (axis permutations in the library's fixed order)
    const int pa[6] = {0, 0, 1, 1, 2, 2}, pb[6] = {1, 2, 0, 2, 0, 1};
    t.off.assign(6 * ne * 3, 0);
    for (int ty = 0; ty < 6; ++ty) {
        int v[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {p, p, p}};
        v[1][pa[ty]] = p;
        v[2][pa[ty]] = p;
        v[2][pb[ty]] = p;
        for (int i = 0; i < ne; ++i) {
            const auto &E = B.ent[i];
            int o[3];
            for (int d = 0; d < 3; ++d) {
                if (E[0] == 0) {
                    o[d] = v[E[1]][d];
                } else if (E[0] == 1) {
                    const int k = E[4];
                    o[d] = v[E[1]][d] + (k + 1) * (v[E[2]][d] - v[E[1]][d]) / p;
                } else if (E[0] == 2) {
                    const int ii = E[4] >> 8, jj = E[4] & 255;
                    o[d] = v[E[1]][d] + ((ii + 1) * (v[E[2]][d] - v[E[1]][d]) + (jj + 1) * (v[E[3]][d] - v[E[1]][d])) / p;
                } else {
                    o[d] = (v[0][d] + v[1][d] + v[2][d] + v[3][d]) / 4;
                }
            }
            for (int d = 0; d < 3; ++d) t.off[(ty * ne + i) * 3 + d] = o[d];
        }
    }
    return true;
}

}  // namespace hp
}  // namespace chom
