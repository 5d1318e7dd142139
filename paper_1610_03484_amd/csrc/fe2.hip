// Fully nested multi-scale run (FE^2, paper Sec. 3 and Sec. 5) on a synthetic
// macro box: macro heat and moisture transport (Eq. Eq_field in the discrete
// form Eq. Eq_field_disc: capacity and conductivity matrices of linear
// elements, implicit Euler in time), the damage of the matrix at every Gauss
// point by the rate form of Sec. 4 (chom_damage_history), an RVE solve at every
// Gauss point with that damage (one batched solve per step), and macro linear
// elasticity with the homogenised stiffnesses.
//
// The macro mesh is the Kuhn lattice of an nx x ny x nz box (six P1 tets per
// cell, one Gauss point -- the centroid -- per tet), so every macro operator is
// a 15-point stencil on the vertex lattice, assembled per vertex by gathering
// over the tets at the vertex (no atomics), C x C blocks per entry.  The macro
// systems are small (thousands of unknowns): each is solved in FP64 by
// Jacobi-preconditioned CG in one workgroup, whose barriers replace kernel
// launches between the CG's phases.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace chom {
namespace {

constexpr int FE_BS = 1024;
constexpr double kFeTgC = 126.0;   // glass transition of the degradation law (Sec. 4), Celsius

struct Box {
    int nx, ny, nz;
    double hx, hy, hz;
    long long nv;
};

__host__ __device__ inline long long bvid(const Box &b, int i, int j, int k) {
    return i + (long long)(b.nx + 1) * (j + (long long)(b.ny + 1) * k);
}

__device__ inline void bxyz(const Box &b, long long v, int &i, int &j, int &k) {
    i = (int)(v % (b.nx + 1));
    j = (int)((v / (b.nx + 1)) % (b.ny + 1));
    k = (int)(v / ((long long)(b.nx + 1) * (b.ny + 1)));
}

// Stencil slot of a Kuhn neighbour offset (-1 if the offset is not one).
__device__ inline int fe_slot(int dx, int dy, int dz) {
    for (int s = 0; s < MG_SLOTS; ++s) {
        int a, b, c;
        kuhn_offset(s, a, b, c);
        if (a == dx && b == dy && c == dz) return s;
    }
    return -1;
}

// Lattice vertices of Kuhn tet t of cell (ci, cj, ck).
__device__ inline void fe_tet(int ci, int cj, int ck, int t, int v[4][3]) {
    int p0, p1;
    kuhn_perm(t, p0, p1);
    for (int a = 0; a < 4; ++a) {
        v[a][0] = ci;
        v[a][1] = cj;
        v[a][2] = ck;
    }
    v[1][p0] += 1;
    v[2][p0] += 1;
    v[2][p1] += 1;
    v[3][0] += 1;
    v[3][1] += 1;
    v[3][2] += 1;
}

// Barycentric gradients and volume of a box tet (vertices at lattice * h).
__device__ inline double fe_grads(const Box &b, const int v[4][3], double g[4][3]) {
    const double h[3] = {b.hx, b.hy, b.hz};
    double J[3][3];   // columns: edges from vertex 0
    for (int d = 0; d < 3; ++d)
        for (int e = 0; e < 3; ++e) J[d][e] = (v[e + 1][d] - v[0][d]) * h[d];
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    const double id = 1.0 / det;
    // rows of J^-1 are the gradients of lambda_1..3
    g[1][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
    g[1][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    g[1][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    g[2][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
    g[2][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    g[2][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    g[3][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
    g[3][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    g[3][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
    return fabs(det) / 6.0;
}

// Scalar transport stencils of vertex v: A = cap/dt M + K and Mdt = cap/dt M,
// M the consistent P1 mass (int N_a N_b = |e| (1 + delta_ab) / 20), K the
// conductivity matrix int grad N_a . Kc grad N_b (Kc [3][3]).
__global__ __launch_bounds__(256) void fe_scalar_assemble_kernel(Box b, const double *Kc, double cap_dt, double *A,
                                                                 double *Mdt) {
    const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (v >= b.nv) return;
    int i, j, k;
    bxyz(b, v, i, j, k);
    double ra[MG_SLOTS], rm[MG_SLOTS];
    for (int s = 0; s < MG_SLOTS; ++s) ra[s] = rm[s] = 0.0;
    double Kl[3][3];
    for (int d = 0; d < 3; ++d)
        for (int e = 0; e < 3; ++e) Kl[d][e] = Kc[d * 3 + e];
    for (int dk = -1; dk <= 0; ++dk)
        for (int dj = -1; dj <= 0; ++dj)
            for (int di = -1; di <= 0; ++di) {
                const int ci = i + di, cj = j + dj, ck = k + dk;
                if (ci < 0 || cj < 0 || ck < 0 || ci >= b.nx || cj >= b.ny || ck >= b.nz) continue;
                for (int t = 0; t < 6; ++t) {
                    int lv[4][3];
                    fe_tet(ci, cj, ck, t, lv);
                    int a = -1;
                    for (int q = 0; q < 4; ++q)
                        if (lv[q][0] == i && lv[q][1] == j && lv[q][2] == k) a = q;
                    if (a < 0) continue;
                    double g[4][3];
                    const double vol = fe_grads(b, lv, g);
                    double kg[3];
                    for (int d = 0; d < 3; ++d) kg[d] = Kl[d][0] * g[a][0] + Kl[d][1] * g[a][1] + Kl[d][2] * g[a][2];
                    for (int q = 0; q < 4; ++q) {
                        const int s = fe_slot(lv[q][0] - i, lv[q][1] - j, lv[q][2] - k);
                        if (s < 0) continue;   // not reached: a Kuhn tet's vertices are Kuhn neighbours
                        const double m = cap_dt * vol * (q == a ? 2.0 : 1.0) / 20.0;
                        ra[s] += vol * (kg[0] * g[q][0] + kg[1] * g[q][1] + kg[2] * g[q][2]) + m;
                        rm[s] += m;
                    }
                }
            }
    for (int s = 0; s < MG_SLOTS; ++s) {
        A[v * MG_SLOTS + s] = ra[s];
        Mdt[v * MG_SLOTS + s] = rm[s];
    }
}

// Elasticity stencil of vertex v: 3 x 3 blocks K_ab = |e| B_a^T C_e B_b summed
// over the tets at v, C_e the tet's homogenised stiffness (21 upper-triangle
// values of the Voigt matrix: stress [11 22 33 12 23 31] from engineering
// strain [11 22 33 2*12 2*23 2*31]).
__global__ __launch_bounds__(256) void fe_elastic_assemble_kernel(Box b, const double *C21, double *A) {
    const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (v >= b.nv) return;
    int i, j, k;
    bxyz(b, v, i, j, k);
    double row[MG_SLOTS][9];
    for (int s = 0; s < MG_SLOTS; ++s)
        for (int e = 0; e < 9; ++e) row[s][e] = 0.0;
    for (int dk = -1; dk <= 0; ++dk)
        for (int dj = -1; dj <= 0; ++dj)
            for (int di = -1; di <= 0; ++di) {
                const int ci = i + di, cj = j + dj, ck = k + dk;
                if (ci < 0 || cj < 0 || ck < 0 || ci >= b.nx || cj >= b.ny || ck >= b.nz) continue;
                const long long cell = ci + (long long)b.nx * (cj + (long long)b.ny * ck);
                for (int t = 0; t < 6; ++t) {
                    int lv[4][3];
                    fe_tet(ci, cj, ck, t, lv);
                    int a = -1;
                    for (int q = 0; q < 4; ++q)
                        if (lv[q][0] == i && lv[q][1] == j && lv[q][2] == k) a = q;
                    if (a < 0) continue;
                    double g[4][3];
                    const double vol = fe_grads(b, lv, g);
                    const double *c21 = C21 + (cell * 6 + t) * 21;
                    double Cm[6][6];
                    for (int r = 0, u = 0; r < 6; ++r)
                        for (int c = r; c < 6; ++c, ++u) Cm[r][c] = Cm[c][r] = c21[u];
                    // B_a^T C: 3 x 6
                    const double *ga = g[a];
                    double BaT[3][6] = {{ga[0], 0, 0, ga[1], 0, ga[2]},
                                        {0, ga[1], 0, ga[0], ga[2], 0},
                                        {0, 0, ga[2], 0, ga[1], ga[0]}};
                    double BC[3][6];
                    for (int r = 0; r < 3; ++r)
                        for (int c = 0; c < 6; ++c) {
                            double sacc = 0.0;
                            for (int m = 0; m < 6; ++m) sacc += BaT[r][m] * Cm[m][c];
                            BC[r][c] = sacc;
                        }
                    for (int q = 0; q < 4; ++q) {
                        const int s = fe_slot(lv[q][0] - i, lv[q][1] - j, lv[q][2] - k);
                        if (s < 0) continue;   // not reached: a Kuhn tet's vertices are Kuhn neighbours
                        const double *gb = g[q];
                        // B_b: 6 x 3
                        const double Bb[6][3] = {{gb[0], 0, 0}, {0, gb[1], 0}, {0, 0, gb[2]},
                                                 {gb[1], gb[0], 0}, {0, gb[2], gb[1]}, {gb[2], 0, gb[0]}};
                        for (int r = 0; r < 3; ++r)
                            for (int c = 0; c < 3; ++c) {
                                double sacc = 0.0;
                                for (int m = 0; m < 6; ++m) sacc += BC[r][m] * Bb[m][c];
                                row[s][r * 3 + c] += vol * sacc;
                            }
                    }
                }
            }
    for (int s = 0; s < MG_SLOTS; ++s)
        for (int e = 0; e < 9; ++e) A[(v * MG_SLOTS + s) * 9 + e] = row[s][e];
}

__device__ inline double fe_block_sum(double v, double *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < nw; ++q) s += red[q];
    return s;
}

// (A x) at unknown (v, c) over the stencil; neighbours outside the box carry
// zero coefficients and are skipped.
template <int C>
__device__ inline double fe_apply(const Box &b, const double *A, const double *x, long long v, int c) {
    int i, j, k;
    bxyz(b, v, i, j, k);
    double s = 0.0;
    for (int t = 0; t < MG_SLOTS; ++t) {
        int dx, dy, dz;
        kuhn_offset(t, dx, dy, dz);
        const int ni = i + dx, nj = j + dy, nk = k + dz;
        if (ni < 0 || nj < 0 || nk < 0 || ni > b.nx || nj > b.ny || nk > b.nz) continue;
        const long long w = bvid(b, ni, nj, nk);
        const double *blk = A + (v * MG_SLOTS + t) * C * C;
        for (int d = 0; d < C; ++d) s += blk[c * C + d] * x[w * C + d];
    }
    return s;
}

// b = Mdt psi (right side of the implicit step).
__global__ __launch_bounds__(256) void fe_mass_rhs_kernel(Box b, const double *Mdt, const double *psi, double *rhs) {
    const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (v >= b.nv) return;
    rhs[v] = fe_apply<1>(b, Mdt, psi, v, 0);
}

// Jacobi-preconditioned CG in one workgroup on A x = rhs: unknowns with
// fixed[u] != 0 keep their value in x (Dirichlet data); the others start from
// x.  Stops when r.z <= rtol2 r0.z0 (or r = 0) or after max_iter steps;
// *iters = steps taken, negated (minus one) if not converged.
template <int C>
__global__ __launch_bounds__(FE_BS) void fe_cg_kernel(Box b, const double *A, const double *rhs, double *x,
                                                      const int *fixed, double *r, double *p, double *q,
                                                      double rtol2, int max_iter, int *iters) {
    __shared__ double red[FE_BS / 64];
    const long long nu = b.nv * C;
    auto diag = [&](long long u) { return A[((u / C) * MG_SLOTS) * C * C + (u % C) * C + (u % C)]; };
    double loc = 0.0;
    for (long long u = threadIdx.x; u < nu; u += blockDim.x) {
        double rv = 0.0;
        if (!fixed[u]) rv = (rhs ? rhs[u] : 0.0) - fe_apply<C>(b, A, x, u / C, (int)(u % C));
        r[u] = rv;
        const double z = fixed[u] ? 0.0 : rv / diag(u);
        p[u] = z;
        loc += rv * z;
    }
    double rz = fe_block_sum(loc, red);
    const double rz0 = rz;
    int it = 0;
    bool conv = rz <= rtol2 * rz0 || rz == 0.0;
    while (!conv && it < max_iter) {
        loc = 0.0;
        for (long long u = threadIdx.x; u < nu; u += blockDim.x) {
            double qv = 0.0;
            if (!fixed[u]) qv = fe_apply<C>(b, A, p, u / C, (int)(u % C));
            q[u] = qv;
            loc += p[u] * qv;
        }
        const double pq = fe_block_sum(loc, red);
        if (!(pq > 0.0)) break;
        const double alpha = rz / pq;
        loc = 0.0;
        for (long long u = threadIdx.x; u < nu; u += blockDim.x) {
            if (fixed[u]) continue;
            x[u] += alpha * p[u];
            const double rv = r[u] - alpha * q[u];
            r[u] = rv;
            loc += rv * rv / diag(u);
        }
        const double rzn = fe_block_sum(loc, red);
        ++it;
        conv = rzn <= rtol2 * rz0;
        const double beta = rzn / rz;
        rz = rzn;
        for (long long u = threadIdx.x; u < nu; u += blockDim.x)
            if (!fixed[u]) p[u] = r[u] / diag(u) + beta * p[u];
        __syncthreads();
    }
    if (threadIdx.x == 0) *iters = conv ? it : -(it + 1);
}

// Gauss-point values (tet means of the vertex values) of T and c.
__global__ __launch_bounds__(256) void fe_gauss_kernel(Box b, const double *T, const double *c, double *Tg,
                                                       double *cg) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long ne = 6LL * b.nx * b.ny * b.nz;
    if (e >= ne) return;
    const int t = (int)(e % 6);
    const long long cell = e / 6;
    const int ci = (int)(cell % b.nx), cj = (int)((cell / b.nx) % b.ny), ck = (int)(cell / ((long long)b.nx * b.ny));
    int lv[4][3];
    fe_tet(ci, cj, ck, t, lv);
    double st = 0.0, sc = 0.0;
    for (int a = 0; a < 4; ++a) {
        const long long v = bvid(b, lv[a][0], lv[a][1], lv[a][2]);
        st += T[v];
        sc += c[v];
    }
    Tg[e] = 0.25 * st;
    cg[e] = 0.25 * sc;
}

// x-force on the face x = lx: the sum of (A u)_x over its vertices (A the full
// stencil, Dirichlet rows included).
__global__ __launch_bounds__(FE_BS) void fe_reaction_kernel(Box b, const double *A, const double *u, double *out) {
    __shared__ double red[FE_BS / 64];
    double loc = 0.0;
    const long long nface = (long long)(b.ny + 1) * (b.nz + 1);
    for (long long f = threadIdx.x; f < nface; f += blockDim.x) {
        const int j = (int)(f % (b.ny + 1)), k = (int)(f / (b.ny + 1));
        loc += fe_apply<3>(b, A, u, bvid(b, b.nx, j, k), 0);
    }
    const double s = fe_block_sum(loc, red);
    if (threadIdx.x == 0) *out = s;
}

template <typename T> struct HostDev {
    std::vector<T> h;
    DevBuf<T> d;
};

int fe2_fail(const std::string &msg, int code) {
    set_error("chom_fe2_run: " + msg);
    return code;
}

}  // namespace
}  // namespace chom

using namespace chom;

extern "C" int chom_fe2_run(chom_rve *rve, const chom_fe2_problem *P, chom_fe2_output *out) {
    if (!rve || !P) return fe2_fail("null handle or problem", CHOM_EINVAL);
    if (P->surrogate && !(P->surrogate_thresh >= 0))
        return fe2_fail("the surrogate's fallback threshold must be >= 0", CHOM_EINVAL);
    if (P->nx < 1 || P->ny < 1 || P->nz < 1 || P->nx > 256 || P->ny > 256 || P->nz > 256 || !(P->lx > 0) ||
        !(P->ly > 0) || !(P->lz > 0) || !(P->heat_capacity > 0) || !(P->dt_years > 0) || P->steps < 1 ||
        !(P->macro_rtol > 0) || P->macro_max_iter < 1 || !std::isfinite(P->strain_x) || !std::isfinite(P->T0) ||
        !std::isfinite(P->c0) || !std::isfinite(P->T_top) || !std::isfinite(P->c_top))
        return fe2_fail("cells in 1..256 per side, positive lengths, capacity, time step, tolerance and caps "
                        "required",
                        CHOM_EINVAL);
    // The degradation law holds below the glass transition and for non-negative
    // moisture (Sec. 4): the initial state and the exposure must lie there.
    if (!(P->T0 < kFeTgC) || !(P->T_top < kFeTgC) || !(P->c0 >= 0) || !(P->c_top >= 0))
        return fe2_fail("initial state and exposure outside the degradation law's domain (T < T_g = 126 C, "
                        "c >= 0)",
                        CHOM_EINVAL);
    Box b;
    b.nx = P->nx;
    b.ny = P->ny;
    b.nz = P->nz;
    b.hx = P->lx / P->nx;
    b.hy = P->ly / P->ny;
    b.hz = P->lz / P->nz;
    b.nv = (long long)(P->nx + 1) * (P->ny + 1) * (P->nz + 1);
    const long long nv = b.nv, ngp = 6LL * P->nx * P->ny * P->nz;
    double factors[8];
    for (int q = 0; q < 8; ++q) factors[q] = P->factors ? P->factors[q] : 1.0;
    double c_sat = 0.0;
    int degrade_yarn = 0;
    rve_settings(rve, &c_sat, &degrade_yarn);
    int status = CHOM_OK;

    // ---- homogenised transport coefficients of the undegraded record (once)
    chom_params p0;
    p0.T_celsius = 20.0;
    p0.c_wt = 0.0;
    p0.t_years = 0.0;
    for (int q = 0; q < 8; ++q) p0.factor[q] = factors[q];
    double C0[21], K0[6], D0[6];
    chom_report rep0;
    int st = rve_homogenise_host(rve, &p0, 1, C0, K0, D0, &rep0);
    if (st != CHOM_OK && st != CHOM_ENOCONV) return st;
    if (st == CHOM_ENOCONV) status = CHOM_ENOCONV;
    auto full3 = [](const double *k6, double *m) {
        const int id[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {1, 2}, {0, 2}};
        for (int q = 0; q < 6; ++q) m[id[q][0] * 3 + id[q][1]] = m[id[q][1] * 3 + id[q][0]] = k6[q];
    };
    double Kt[9], Dc[9];
    full3(K0, Kt);
    full3(D0, Dc);

    hipStream_t s = nullptr;
    CHOM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() {
            if (s) (void)hipStreamDestroy(s);
        }
    } guard{s};

    DevBuf<double> kt, dc, At, Mt, Ac, Mc, Au, T, c, rhs, u, r, p, q, Tg, cg, C21, react;
    DevBuf<int> fix1, fix3, its;
    CHOM_HIP(kt.ensure(9));
    CHOM_HIP(dc.ensure(9));
    CHOM_HIP(At.ensure((size_t)nv * MG_SLOTS));
    CHOM_HIP(Mt.ensure((size_t)nv * MG_SLOTS));
    CHOM_HIP(Ac.ensure((size_t)nv * MG_SLOTS));
    CHOM_HIP(Mc.ensure((size_t)nv * MG_SLOTS));
    CHOM_HIP(Au.ensure((size_t)nv * MG_SLOTS * 9));
    CHOM_HIP(T.ensure((size_t)nv));
    CHOM_HIP(c.ensure((size_t)nv));
    CHOM_HIP(rhs.ensure((size_t)nv));
    CHOM_HIP(u.ensure((size_t)nv * 3));
    CHOM_HIP(r.ensure((size_t)nv * 3));
    CHOM_HIP(p.ensure((size_t)nv * 3));
    CHOM_HIP(q.ensure((size_t)nv * 3));
    CHOM_HIP(Tg.ensure((size_t)ngp));
    CHOM_HIP(cg.ensure((size_t)ngp));
    CHOM_HIP(C21.ensure((size_t)ngp * 21));
    CHOM_HIP(react.ensure(1));
    CHOM_HIP(fix1.ensure((size_t)nv));
    CHOM_HIP(fix3.ensure((size_t)nv * 3));
    CHOM_HIP(its.ensure(3));

    // ---- Dirichlet data: T, c on z = lz; u_x on x = 0 and x = lx, u_y on y = 0, u_z on z = 0
    std::vector<int> hf1(nv), hf3(nv * 3);
    std::vector<double> hT(nv, P->T0), hc(nv, P->c0), hu(nv * 3, 0.0);
    for (int k = 0; k <= P->nz; ++k)
        for (int j = 0; j <= P->ny; ++j)
            for (int i = 0; i <= P->nx; ++i) {
                const long long v = bvid(b, i, j, k);
                hf1[v] = k == P->nz;
                hf3[v * 3 + 0] = i == 0 || i == P->nx;
                hf3[v * 3 + 1] = j == 0;
                hf3[v * 3 + 2] = k == 0;
                if (i == P->nx) hu[v * 3] = P->strain_x * P->lx;
            }
    CHOM_HIP(hipMemcpyAsync(fix1.p, hf1.data(), sizeof(int) * nv, hipMemcpyHostToDevice, s));
    CHOM_HIP(hipMemcpyAsync(fix3.p, hf3.data(), sizeof(int) * nv * 3, hipMemcpyHostToDevice, s));
    CHOM_HIP(hipMemcpyAsync(T.p, hT.data(), sizeof(double) * nv, hipMemcpyHostToDevice, s));
    CHOM_HIP(hipMemcpyAsync(c.p, hc.data(), sizeof(double) * nv, hipMemcpyHostToDevice, s));
    CHOM_HIP(hipMemcpyAsync(kt.p, Kt, sizeof(double) * 9, hipMemcpyHostToDevice, s));
    CHOM_HIP(hipMemcpyAsync(dc.p, Dc, sizeof(double) * 9, hipMemcpyHostToDevice, s));
    const int gv = (int)((nv + 255) / 256), gg = (int)((ngp + 255) / 256);
    fe_scalar_assemble_kernel<<<gv, 256, 0, s>>>(b, kt.p, P->heat_capacity / P->dt_years, At.p, Mt.p);
    fe_scalar_assemble_kernel<<<gv, 256, 0, s>>>(b, dc.p, 1.0 / P->dt_years, Ac.p, Mc.p);
    CHOM_HIP(hipGetLastError());
    if (out && out->T) std::memcpy(out->T, hT.data(), sizeof(double) * nv);
    if (out && out->c) std::memcpy(out->c, hc.data(), sizeof(double) * nv);
    if (out) {
        out->macro_iters[0] = out->macro_iters[1] = out->macro_iters[2] = 0;
        out->n_fallback = 0;
    }
    // with a surrogate whose arrays live on the device, the Gauss-point records
    // and results pass through device buffers
    const bool sur_dev = P->surrogate && mlp_device_ptrs(P->surrogate);
    DevBuf<double> sp, sC, sK, sD;
    if (sur_dev) {
        CHOM_HIP(sp.ensure((size_t)ngp * 11));
        CHOM_HIP(sC.ensure((size_t)ngp * 21));
        CHOM_HIP(sK.ensure((size_t)ngp * 6));
        CHOM_HIP(sD.ensure((size_t)ngp * 6));
    }

    std::vector<double> hkeep(ngp, 1.0), hTg(ngp), hcg(ngp), hfac(ngp * 8), hC(ngp * 21), hK(ngp * 6), hD(ngp * 6);
    std::vector<chom_params> hpar(ngp);
    std::vector<chom_report> hrep(ngp);
    for (long long e = 0; e < ngp; ++e)
        for (int qq = 0; qq < 8; ++qq) hfac[e * 8 + qq] = factors[qq];
    const double rtol2 = P->macro_rtol * P->macro_rtol;
    const double dt = P->dt_years;
    for (int step = 0; step < P->steps; ++step) {
        // ---- heat and moisture: (cap/dt M + K) psi^{n+1} = cap/dt M psi^n, Dirichlet top values
        int hits[3];
        for (int phys = 0; phys < 2; ++phys) {
            DevBuf<double> &F = phys == 0 ? T : c;
            const double *A = phys == 0 ? At.p : Ac.p;
            const double *M = phys == 0 ? Mt.p : Mc.p;
            fe_mass_rhs_kernel<<<gv, 256, 0, s>>>(b, M, F.p, rhs.p);
            // impose the face value on the previous field (the free values are the start)
            const double top = phys == 0 ? P->T_top : P->c_top;
            std::vector<double> &hF = phys == 0 ? hT : hc;
            CHOM_HIP(hipMemcpyAsync(hF.data(), F.p, sizeof(double) * nv, hipMemcpyDeviceToHost, s));
            CHOM_HIP(hipStreamSynchronize(s));
            for (long long v = 0; v < nv; ++v)
                if (hf1[v]) hF[v] = top;
            CHOM_HIP(hipMemcpyAsync(F.p, hF.data(), sizeof(double) * nv, hipMemcpyHostToDevice, s));
            fe_cg_kernel<1><<<1, FE_BS, 0, s>>>(b, A, rhs.p, F.p, fix1.p, r.p, p.p, q.p, rtol2, P->macro_max_iter,
                                                its.p + phys);
        }
        fe_gauss_kernel<<<gg, 256, 0, s>>>(b, T.p, c.p, Tg.p, cg.p);
        CHOM_HIP(hipGetLastError());
        CHOM_HIP(hipMemcpyAsync(hTg.data(), Tg.p, sizeof(double) * ngp, hipMemcpyDeviceToHost, s));
        CHOM_HIP(hipMemcpyAsync(hcg.data(), cg.p, sizeof(double) * ngp, hipMemcpyDeviceToHost, s));
        CHOM_HIP(hipMemcpyAsync(hits, its.p, sizeof(int) * 2, hipMemcpyDeviceToHost, s));
        CHOM_HIP(hipStreamSynchronize(s));
        // ---- damage at every Gauss point (implicit Euler over this step) and its equivalent record
        std::vector<double> knew(ngp);
        st = chom_damage_history(ngp, 1, hTg.data(), hcg.data(), &dt, hkeep.data(), hfac.data(), c_sat, 0, s,
                                 knew.data(), hpar.data());
        if (st != CHOM_OK) return st;
        hkeep = knew;
        // ---- the RVE (or the surrogate with the RVE as fallback) at every Gauss point
        if (P->surrogate) {
            int64_t nfb = 0;
            if (sur_dev) {
                CHOM_HIP(hipMemcpy(sp.p, hpar.data(), sizeof(double) * ngp * 11, hipMemcpyHostToDevice));
                st = chom_homogenise_surrogate(P->surrogate, rve, reinterpret_cast<const chom_params *>(sp.p), ngp,
                                               P->surrogate_thresh, 0, sC.p, sK.p, sD.p, nullptr, nullptr, &nfb);
                if (st == CHOM_OK || st == CHOM_ENOCONV) {
                    CHOM_HIP(hipMemcpy(hC.data(), sC.p, sizeof(double) * ngp * 21, hipMemcpyDeviceToHost));
                    CHOM_HIP(hipMemcpy(hK.data(), sK.p, sizeof(double) * ngp * 6, hipMemcpyDeviceToHost));
                    CHOM_HIP(hipMemcpy(hD.data(), sD.p, sizeof(double) * ngp * 6, hipMemcpyDeviceToHost));
                }
            } else {
                st = chom_homogenise_surrogate(P->surrogate, rve, hpar.data(), ngp, P->surrogate_thresh, 0, hC.data(),
                                               hK.data(), hD.data(), nullptr, nullptr, &nfb);
            }
            if (out) out->n_fallback += nfb;
        } else {
            st = rve_homogenise_host(rve, hpar.data(), (int)ngp, hC.data(), hK.data(), hD.data(), hrep.data());
        }
        if (st == CHOM_ENOCONV) status = CHOM_ENOCONV;
        else if (st != CHOM_OK) return st;
        // ---- macro elasticity
        CHOM_HIP(hipMemcpyAsync(C21.p, hC.data(), sizeof(double) * ngp * 21, hipMemcpyHostToDevice, s));
        // the previous step's displacement (same Dirichlet data) starts the solve
        if (step == 0) CHOM_HIP(hipMemcpyAsync(u.p, hu.data(), sizeof(double) * nv * 3, hipMemcpyHostToDevice, s));
        fe_elastic_assemble_kernel<<<gv, 256, 0, s>>>(b, C21.p, Au.p);
        fe_cg_kernel<3><<<1, FE_BS, 0, s>>>(b, Au.p, nullptr, u.p, fix3.p, r.p, p.p, q.p, rtol2, P->macro_max_iter,
                                            its.p + 2);
        fe_reaction_kernel<<<1, FE_BS, 0, s>>>(b, Au.p, u.p, react.p);
        CHOM_HIP(hipGetLastError());
        double R = 0.0;
        CHOM_HIP(hipMemcpyAsync(&R, react.p, sizeof(double), hipMemcpyDeviceToHost, s));
        CHOM_HIP(hipMemcpyAsync(&hits[2], its.p + 2, sizeof(int), hipMemcpyDeviceToHost, s));
        if (out && out->T) CHOM_HIP(hipMemcpyAsync(out->T + (size_t)(step + 1) * nv, T.p, sizeof(double) * nv,
                                                   hipMemcpyDeviceToHost, s));
        if (out && out->c) CHOM_HIP(hipMemcpyAsync(out->c + (size_t)(step + 1) * nv, c.p, sizeof(double) * nv,
                                                   hipMemcpyDeviceToHost, s));
        if (out && out->u && step == P->steps - 1)
            CHOM_HIP(hipMemcpyAsync(out->u, u.p, sizeof(double) * nv * 3, hipMemcpyDeviceToHost, s));
        CHOM_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < 3; ++k) {
            if (hits[k] < 0) status = CHOM_ENOCONV;
            const int itk = hits[k] < 0 ? -hits[k] - 1 : hits[k];
            if (out) out->macro_iters[k] = std::max(out->macro_iters[k], itk);
        }
        if (out && out->reaction) out->reaction[step] = R;
        if (out && out->keep) std::memcpy(out->keep + (size_t)step * ngp, hkeep.data(), sizeof(double) * ngp);
        if (out && out->C_bar && step == P->steps - 1) std::memcpy(out->C_bar, hC.data(), sizeof(double) * ngp * 21);
    }
    if (status == CHOM_ENOCONV) set_error("chom_fe2_run: a macro or RVE solve did not converge (outputs written)");
    return status;
}
