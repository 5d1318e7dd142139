// Internal definitions shared by the HIP sources of libchom.
//
// Discretisation used on the device: the RVE is the Kuhn lattice of an n^3 grid
// and the order-2 hierarchic space on it (vertex functions lam_a, edge functions
// 4 lam_a lam_b; the paper's hierarchic basis, Sec. 1 and Sec. 7).  Every
// degree of freedom sits on a point of the (2n+1)^3 lattice: a vertex at even
// coordinates, an edge at the sum of its end points' grid coordinates, so the
// DOF number is the lattice index and no connectivity is stored.  Because the
// vertices of every Kuhn tet are listed in increasing global id, the local
// vertex order is the global one and all entity orientations agree between
// neighbouring tets and across periodic faces.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chom {

// Operator tile: TX x TY x TZ cells per workgroup; its DOF box is (2T+1)^3.
// One thread per tet of the tile (192 threads).
constexpr int TX = 4, TY = 4, TZ = 2;
constexpr int BX = 2 * TX + 1, BY = 2 * TY + 1, BZ = 2 * TZ + 1;
constexpr int BOXPTS = BX * BY * BZ;
constexpr int TILE_TETS = 6 * TX * TY * TZ;

// Per-RVE geometry.  Kernels read it from a device array, indexed by the
// problem's `geo`, so one launch can mix RVEs of different sizes and BCs.
struct Geo {
    int n;            // cells per side
    int bc;           // 0 Dirichlet, 1 periodic, 2 Neumann
    int uniform;      // 1: undistorted grid, geometry from the six tet types
    int Lw;           // stored lattice points per side: 2n (periodic) or 2n+1
    long long npts;   // Lw^3
    double volume;    // RVE volume
    double tg64[6][10];   // uniform: per tet type grad(lam_1..3) (9) and volume
    float tg32[6][10];
    const double4 *elem64;  // per tet: fibre axis xyz, phase in w
    const float4 *elem32;
    const double *geo64;    // non-uniform: per tet grad(lam_1..3) (9) and volume
    const float *geo32;
    const double *rows;     // per lattice point: int grad(phi) (3) and int phi (1)
    int nrow;               // projection rows per component: 0 (D), 1 (P), 4 (N)
    int tiles_x, tiles_y, tiles_z;
    int ntiles;       // operator tiles (order 2: TX x TY x TZ cells; orders 3, 4: one cell)
    int tcx, tcy, tcz;        // cells per operator tile along each axis
    int bx, by, bz, boxpts;   // DOF box of a tile: p tc + 1 points per axis
    int p;            // polynomial order
    int L;            // lattice points per side minus one: p n
    // orders 3, 4: basis tables (see hp_tables.cpp)
    const int *hoff;                 // [6][ne][3] lattice offset of each local DOF per tet type
    const double *hW, *hWd, *hSd;    // [ne], [3][ne], [9][ne]
    const double *hDA64, *hDB64;     // padded [D_1; D_2; D_3] and its transpose
    const float *hDA32, *hDB32;
    // P1 coarse hierarchy of the two-level preconditioner (see mg.hip): level 0
    // is the vertex lattice (the vertex functions of the hierarchic basis are the
    // P1 hats), level l + 1 halves the cells of level l.  mg_nlev = 0: none.
    int mg_nlev;
    int mg_n[8];              // cells per side of level l
    int mg_lw[8];             // stored points per side: n_l (periodic) or n_l + 1
    long long mg_off[8];      // first point of level l within the RVE's coarse points
    long long mg_pts;         // coarse points over all levels
    // index tables of the coarse levels, [mg_off[l] + point][16] (built on the host):
    const int *mg_nbr;        // the 15 stencil neighbours (the point itself outside the lattice,
                              // where the stencil block is zero)
    const int *mg_child;      // l >= 1: the 15 children on level l - 1 (-1: none); level 1:
                              // fine lattice indices of the children (-1: none or Dirichlet)
    const int *mg_par;        // l < nlev - 1: the two parents on level l + 1 (equal for an even point)
};

// Kuhn neighbours of a lattice point (the P1 stencil): itself, the seven edge
// directions of the Kuhn split, and their opposites (slot k + 7 = -slot k).
__host__ __device__ inline void kuhn_offset(int k, int &dx, int &dy, int &dz) {
    const int ox[8] = {0, 1, 0, 0, 1, 1, 0, 1};
    const int oy[8] = {0, 0, 1, 0, 1, 0, 1, 1};
    const int oz[8] = {0, 0, 0, 1, 0, 1, 1, 1};
    const int b = k < 8 ? k : k - 7;
    const int sg = k < 8 ? 1 : -1;
    dx = sg * ox[b];
    dy = sg * oy[b];
    dz = sg * oz[b];
}
constexpr int MG_SLOTS = 15;
constexpr int MG_MAXLEV = 8;

// Coarse-correction operands of the CG direction kernel (two-level preconditioner).
template <typename T> struct MgDir {
    const T *x0;   // coarse correction f on the n/2 grid, inside vectors [moff * R * C][R][mg_pts][C]
    const T *W;    // unused by the direction kernel
    int on;
};

// Per-problem descriptor (one parameter record x one physics of one RVE).
struct Prob {
    double mat64[2][5];   // [phase 0 matrix, 1 yarn][invariants]
    float mat32[2][5];
    long long voff;       // offset of this problem's vector segment (values)
    long long doff;       // offset of its per-point preconditioner data (points)
    long long qoff;       // offset of its operator tile boxes (values)
    long long eoff;       // orders 3, 4: offset of its element factors (values)
    long long moff;       // offset of its coarse-hierarchy points (two-level preconditioner)
    int geo;              // index of its RVE geometry
    int mg_sweeps;        // coarsest-level sweeps of the two-level preconditioner (0: the class's count)
    double rtol2_scale;   // factor on every rtol^2 of the problem's stopping tests (0: 1)
};

// First constraint row used by a BC: periodic uses only int(phi) (row 3).
__host__ __device__ inline int row_first(int nrow) { return nrow == 1 ? 3 : 0; }

// Kuhn tet type t: axis permutation (p0, p1, p2) in the fixed order.
__host__ __device__ inline void kuhn_perm(int t, int &p0, int &p1) {
    // (0,1,2),(0,2,1),(1,0,2),(1,2,0),(2,0,1),(2,1,0)
    const int a[6] = {0, 0, 1, 1, 2, 2};
    const int b[6] = {1, 2, 0, 2, 0, 1};
    p0 = a[t];
    p1 = b[t];
}

// Local edge list (a < b) and the edge index of a vertex pair.
__host__ __device__ inline int edge_of(int a, int b) {
    // (0,1)->0 (0,2)->1 (0,3)->2 (1,2)->3 (1,3)->4 (2,3)->5
    if (a > b) { int t = a; a = b; b = t; }
    return a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
}
__host__ __device__ inline void edge_verts(int e, int &a, int &b) {
    const int ea[6] = {0, 0, 0, 1, 1, 2};
    const int eb[6] = {1, 2, 3, 2, 3, 3};
    a = ea[e];
    b = eb[e];
}

// Lattice offsets (in units of the p = 2 lattice) of the 10 DOFs of tet type t,
// relative to 2 * (cell origin).  Vertices first (0..3), then edges 0..5.
__host__ __device__ inline void p2_dof_offsets(int t, int off[10][3]) {
    int p0, p1;
    kuhn_perm(t, p0, p1);
    int v[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {2, 2, 2}};
    v[1][p0] = 2;
    v[2][p0] = 2;
    v[2][p1] = 2;
    for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d) off[a][d] = v[a][d];
    for (int e = 0; e < 6; ++e) {
        int a, b;
        edge_verts(e, a, b);
        for (int d = 0; d < 3; ++d) off[4 + e][d] = (v[a][d] + v[b][d]) / 2;
    }
}

// ----------------------------------------------------------------- constitutive laws
// Transversely isotropic stiffness in invariant form with unit axis a:
//   sigma = lam tr(e) I + 2 muT e + alpha ((a.e.a) I + tr(e) a a) + 2 dmu (a (e a) + (e a) a)
//         + beta (a.e.a) a a.
// e and s are tensor components (xx, yy, zz, xy, yz, zx).  With alpha = dmu =
// beta = 0 this is the isotropic Lame law.
template <typename T>
__host__ __device__ inline void stress_ti(const T e[6], const T a[3], const T m[5], T s[6]) {
    const T lam = m[0], muT = m[1], alpha = m[2], dmu = m[3], beta = m[4];
    const T tr = e[0] + e[1] + e[2];
    const T w0 = e[0] * a[0] + e[3] * a[1] + e[5] * a[2];
    const T w1 = e[3] * a[0] + e[1] * a[1] + e[4] * a[2];
    const T w2 = e[5] * a[0] + e[4] * a[1] + e[2] * a[2];
    const T aea = a[0] * w0 + a[1] * w1 + a[2] * w2;
    const T iso = lam * tr + alpha * aea;
    const T c1 = alpha * tr + beta * aea;
    const T tm = T(2) * muT, td = T(2) * dmu;
    s[0] = iso + tm * e[0] + c1 * a[0] * a[0] + T(2) * td * a[0] * w0;
    s[1] = iso + tm * e[1] + c1 * a[1] * a[1] + T(2) * td * a[1] * w1;
    s[2] = iso + tm * e[2] + c1 * a[2] * a[2] + T(2) * td * a[2] * w2;
    s[3] = tm * e[3] + c1 * a[0] * a[1] + td * (a[0] * w1 + w0 * a[1]);
    s[4] = tm * e[4] + c1 * a[1] * a[2] + td * (a[1] * w2 + w1 * a[2]);
    s[5] = tm * e[5] + c1 * a[2] * a[0] + td * (a[2] * w0 + w2 * a[0]);
}

// Transversely isotropic second-order tensor kT I + dk a a applied to g.
template <typename T>
__host__ __device__ inline void flux_ti(const T g[3], const T a[3], const T m[5], T q[3]) {
    const T ag = a[0] * g[0] + a[1] * g[1] + a[2] * g[2];
    const T c = m[1] * ag;
    q[0] = m[0] * g[0] + c * a[0];
    q[1] = m[0] * g[1] + c * a[1];
    q[2] = m[0] * g[2] + c * a[2];
}

// ----------------------------------------------------------------- P2 element kernel
// y = K_e u for one load case on one tet, for the order-2 hierarchic basis.
// g[4][3]: gradients of the barycentric coordinates; vol: |tet|.
// The gradient of u is linear, so strain and stress are linear and fixed by
// their values at the four vertices; the element integrals are then exact:
//   y_a  = int sigma g_a          = vol/4 * S g_a,                 S = sum_c sigma_c
//   y_ab = int sigma 4(l_a g_b + l_b g_a) = 4 (s_a g_b + s_b g_a), s_a = vol/20 (S + sigma_a).
template <typename T, int C>
__host__ __device__ inline void p2_apply(const T g[4][3], T vol, const T a[3], const T m[5],
                                const T u[10][C], T y[10][C]) {
    if constexpr (C == 3) {
        T G0[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                G0[i][j] = u[0][i] * g[0][j] + u[1][i] * g[1][j] + u[2][i] * g[2][j] + u[3][i] * g[3][j];
        T sig[4][6];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            T G[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) G[i][j] = G0[i][j];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (b == c) continue;
                const int e = edge_of(c, b);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const T ue = T(4) * u[4 + e][i];
#pragma unroll
                    for (int j = 0; j < 3; ++j) G[i][j] += ue * g[b][j];
                }
            }
            T eps[6] = {G[0][0], G[1][1], G[2][2], T(0.5) * (G[0][1] + G[1][0]),
                        T(0.5) * (G[1][2] + G[2][1]), T(0.5) * (G[2][0] + G[0][2])};
            stress_ti<T>(eps, a, m, sig[c]);
        }
        T S[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) S[k] = sig[0][k] + sig[1][k] + sig[2][k] + sig[3][k];
        const T v4 = vol * T(0.25), v20 = vol * T(0.05);
#pragma unroll
        for (int a2 = 0; a2 < 4; ++a2) {
            const T *gg = g[a2];
            y[a2][0] = v4 * (S[0] * gg[0] + S[3] * gg[1] + S[5] * gg[2]);
            y[a2][1] = v4 * (S[3] * gg[0] + S[1] * gg[1] + S[4] * gg[2]);
            y[a2][2] = v4 * (S[5] * gg[0] + S[4] * gg[1] + S[2] * gg[2]);
        }
        T s[4][6];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int k = 0; k < 6; ++k) s[c][k] = v20 * (S[k] + sig[c][k]);
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            int a2, b2;
            edge_verts(e, a2, b2);
            const T *ga = g[a2], *gb = g[b2];
            const T *sa = s[a2], *sb = s[b2];
            y[4 + e][0] = T(4) * (sa[0] * gb[0] + sa[3] * gb[1] + sa[5] * gb[2] + sb[0] * ga[0] + sb[3] * ga[1] + sb[5] * ga[2]);
            y[4 + e][1] = T(4) * (sa[3] * gb[0] + sa[1] * gb[1] + sa[4] * gb[2] + sb[3] * ga[0] + sb[1] * ga[1] + sb[4] * ga[2]);
            y[4 + e][2] = T(4) * (sa[5] * gb[0] + sa[4] * gb[1] + sa[2] * gb[2] + sb[5] * ga[0] + sb[4] * ga[1] + sb[2] * ga[2]);
        }
    } else {
        T G0[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) G0[j] = u[0][0] * g[0][j] + u[1][0] * g[1][j] + u[2][0] * g[2][j] + u[3][0] * g[3][j];
        T q[4][3];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            T G[3] = {G0[0], G0[1], G0[2]};
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (b == c) continue;
                const T ue = T(4) * u[4 + edge_of(c, b)][0];
#pragma unroll
                for (int j = 0; j < 3; ++j) G[j] += ue * g[b][j];
            }
            flux_ti<T>(G, a, m, q[c]);
        }
        T S[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) S[k] = q[0][k] + q[1][k] + q[2][k] + q[3][k];
        const T v4 = vol * T(0.25), v20 = vol * T(0.05);
#pragma unroll
        for (int a2 = 0; a2 < 4; ++a2) y[a2][0] = v4 * (S[0] * g[a2][0] + S[1] * g[a2][1] + S[2] * g[a2][2]);
        T s[4][3];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int k = 0; k < 3; ++k) s[c][k] = v20 * (S[k] + q[c][k]);
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            int a2, b2;
            edge_verts(e, a2, b2);
            y[4 + e][0] = T(4) * (s[a2][0] * g[b2][0] + s[a2][1] * g[b2][1] + s[a2][2] * g[b2][2] +
                                  s[b2][0] * g[a2][0] + s[b2][1] * g[a2][1] + s[b2][2] * g[a2][2]);
        }
    }
}

// Element geometry of global tet id `tet` (type t): gradients of lam_0..3 and volume.
template <typename T> struct GeoSel;
template <> struct GeoSel<double> {
    __device__ static inline void get(const Geo &G, long long tet, int t, double g[4][3], double &vol) {
        const double *src = G.uniform ? G.tg64[t] : G.geo64 + tet * 10;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) g[i + 1][j] = src[3 * i + j];
        vol = src[9];
#pragma unroll
        for (int j = 0; j < 3; ++j) g[0][j] = -(g[1][j] + g[2][j] + g[3][j]);
    }
    __device__ static inline void elem(const Geo &G, long long tet, double a[3], int &phase) {
        const double4 v = G.elem64[tet];
        a[0] = v.x; a[1] = v.y; a[2] = v.z;
        phase = (int)v.w;
    }
};
template <> struct GeoSel<float> {
    __device__ static inline void get(const Geo &G, long long tet, int t, float g[4][3], float &vol) {
        const float *src = G.uniform ? G.tg32[t] : G.geo32 + tet * 10;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) g[i + 1][j] = src[3 * i + j];
        vol = src[9];
#pragma unroll
        for (int j = 0; j < 3; ++j) g[0][j] = -(g[1][j] + g[2][j] + g[3][j]);
    }
    __device__ static inline void elem(const Geo &G, long long tet, float a[3], int &phase) {
        const float4 v = G.elem32[tet];
        a[0] = v.x; a[1] = v.y; a[2] = v.z;
        phase = (int)v.w;
    }
};

template <typename T> __device__ inline const T *prob_mat(const Prob &P, int phase);
template <> __device__ inline const double *prob_mat<double>(const Prob &P, int phase) { return P.mat64[phase ? 1 : 0]; }
template <> __device__ inline const float *prob_mat<float>(const Prob &P, int phase) { return P.mat32[phase ? 1 : 0]; }

// Lattice index of DOF point (X, Y, Z) in [0, p n]^3 for the stored layout.
__device__ inline long long lat_index(const Geo &G, int X, int Y, int Z) {
    if (G.bc == 1) {
        const int m = G.L;
        if (X == m) X = 0;
        if (Y == m) Y = 0;
        if (Z == m) Z = 0;
    }
    return (long long)X + (long long)G.Lw * ((long long)Y + (long long)G.Lw * Z);
}

__device__ inline bool dirichlet_boundary(const Geo &G, int X, int Y, int Z) {
    const int m = G.L;
    return G.bc == 0 && (X == 0 || Y == 0 || Z == 0 || X == m || Y == m || Z == m);
}

// Acoustic tensor Q(w)_cd = sum_kl C_ckdl w_k w_l from the stress law.
__device__ inline void acoustic(const double w[3], const double a[3], const double *m, double Q[3][3]) {
    for (int d = 0; d < 3; ++d) {
        double e[6] = {0, 0, 0, 0, 0, 0};
        // sym(e_d (x) w)
        double G3[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int l = 0; l < 3; ++l) G3[d][l] = w[l];
        e[0] = G3[0][0];
        e[1] = G3[1][1];
        e[2] = G3[2][2];
        e[3] = 0.5 * (G3[0][1] + G3[1][0]);
        e[4] = 0.5 * (G3[1][2] + G3[2][1]);
        e[5] = 0.5 * (G3[2][0] + G3[0][2]);
        double s[6];
        stress_ti<double>(e, a, m, s);
        Q[0][d] = s[0] * w[0] + s[3] * w[1] + s[5] * w[2];
        Q[1][d] = s[3] * w[0] + s[1] * w[1] + s[4] * w[2];
        Q[2][d] = s[5] * w[0] + s[4] * w[1] + s[2] * w[2];
    }
}

// Operator output layout: one (p T + 1)^3 box of values per tile and load case
// ("tile boxes"): [tile][load-case group][load case of the group][box point][C],
// so a wave gathering one load case reads contiguous values.  A lattice point on
// a tile face lies in up to two tiles per axis; its value is the sum of its copies.
// Candidate (tile, local) pairs of coordinate X along one axis.
__device__ inline int tile_cands(int X, int T2, int ntiles, int m2, bool per, int tl[2], int lc[2]) {
    int t = (T2 & (T2 - 1)) == 0 ? (X >> (31 - __clz(T2))) : X / T2;   // order 2: T2 = 8, 8, 4
    if (t > ntiles - 1) t = ntiles - 1;
    int k = 0;
    tl[k] = t;
    lc[k] = X - t * T2;
    ++k;
    if (lc[0] == 0 && t > 0) {
        tl[k] = t - 1;
        lc[k] = T2;
        ++k;
    } else if (X == 0 && per) {  // X = 0 is also the top face X = 2n of the last tile
        tl[k] = ntiles - 1;
        lc[k] = m2 - (ntiles - 1) * T2;
        ++k;
    }
    return k;
}

// Sum of the tile-box copies of lattice point (X, Y, Z) for load case w (C
// values).  Tile boxes are [tile][group][box point][rg * C], rg load cases per
// group, R / rg groups.
template <typename T, int C, int R>
__device__ inline void gather_tiles_col(const Geo &G, const T *qt, int rg, int X, int Y, int Z, int w, double out[C]) {
    const int ng = R / rg;
    const int grp = w / rg, rr = w - grp * rg;
    const bool per = (G.bc == 1);
    const int m2 = G.L;
    int tx[2], ty[2], tz[2], lx[2], ly[2], lz[2];
    const int nx = tile_cands(X, G.p * G.tcx, G.tiles_x, m2, per, tx, lx);
    const int ny = tile_cands(Y, G.p * G.tcy, G.tiles_y, m2, per, ty, ly);
    const int nz = tile_cands(Z, G.p * G.tcz, G.tiles_z, m2, per, tz, lz);
    // all (up to eight) copies are loaded before any is summed, so their
    // latencies overlap (zeroed first: no register write waits on a load)
    T cp[8][C];
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int v = 0; v < C; ++v) cp[k][v] = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (a < nx && b < ny && c < nz) {
                    // 32-bit: one problem's tile boxes hold fewer than 2^31 values (checked at setup)
                    const int tile = tx[a] + G.tiles_x * (ty[b] + G.tiles_y * tz[c]);
                    const int off = (((tile * ng + grp) * rg + rr) * G.boxpts + lx[a] + G.bx * (ly[b] + G.by * lz[c])) * C;
#pragma unroll
                    for (int v = 0; v < C; ++v) cp[4 * a + 2 * b + c][v] = qt[off + v];
                }
            }
#pragma unroll
    for (int v = 0; v < C; ++v) {
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) sum += (double)cp[k][v];
        out[v] = sum;
    }
}

// Lattice coordinates of point pt (32-bit arithmetic: a lattice holds fewer than 2^31 points).
__device__ inline void lattice_xyz(const Geo &G, long long pt, int &X, int &Y, int &Z) {
    const int q = (int)pt, lw = G.Lw;
    const int t = q / lw;
    X = q - t * lw;
    Z = t / lw;
    Y = t - Z * lw;
}

// Symmetric point block (packed xx, yy, zz, xy, yz, xz; one entry for C = 1) times v.
template <typename T, int C>
__device__ inline void minv_apply(const T *Mi, const T v[C], T out[C]) {
    if constexpr (C == 3) {
        out[0] = Mi[0] * v[0] + Mi[3] * v[1] + Mi[5] * v[2];
        out[1] = Mi[3] * v[0] + Mi[1] * v[1] + Mi[4] * v[2];
        out[2] = Mi[5] * v[0] + Mi[4] * v[1] + Mi[2] * v[2];
    } else {
        out[0] = Mi[0] * v[0];
    }
}

// Constraint row functions of lattice point pt (the BC's rows, see Geo.rows).
template <int NR>
__device__ inline void load_rows(const Geo &G, long long pt, double row[4]) {
    row[0] = row[1] = row[2] = row[3] = 0.0;
    if constexpr (NR > 0) {
        if (G.nrow > 0) {
            // the point's four row values in one 32-byte access (rows is 256-byte aligned)
            const double4 v = reinterpret_cast<const double4 *>(G.rows)[pt];
            if (G.nrow == 1) {   // periodic: int(phi) only (row_first)
                row[0] = v.w;
            } else {
                row[0] = v.x;
                if constexpr (NR >= 4) {
                    row[1] = v.y;
                    row[2] = v.z;
                    row[3] = v.w;
                }
            }
        }
    }
}

// In-place Gauss-Jordan with partial pivoting on the augmented S x 2S system
// [A | I] (S <= 12) by a whole workgroup (blockDim.x >= 144; every thread
// calls it; `sh` is two ints of LDS): on success the right half holds A^-1;
// returns 0 if singular.  Per pivot one thread picks the row, then the threads
// update one or two entries each between barriers.
__device__ inline int gauss_jordan_wg(double A[12][24], int S, int *sh) {
    const int tid = threadIdx.x, nt = blockDim.x, W = 2 * S;
    for (int c = 0; c < S; ++c) {
        if (tid == 0) {
            int piv = c;
            for (int r = c + 1; r < S; ++r)
                if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
            sh[0] = piv;
            sh[1] = fabs(A[piv][c]) > 0.0 ? 1 : 0;
        }
        __syncthreads();
        if (!sh[1]) return 0;
        const int piv = sh[0];
        if (piv != c) {
            for (int k = tid; k < W; k += nt) {
                const double t = A[c][k];
                A[c][k] = A[piv][k];
                A[piv][k] = t;
            }
            __syncthreads();
        }
        const double ip = 1.0 / A[c][c];
        double nv[2], fv[2];
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int e = tid + m * nt;
            nv[m] = fv[m] = 0.0;
            if (e < S * W) {
                const int r = e / W, k = e - (e / W) * W;
                nv[m] = A[c][k] * ip;
                fv[m] = (r == c) ? 0.0 : A[r][c];
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int e = tid + m * nt;
            if (e < S * W) {
                const int r = e / W, k = e - (e / W) * W;
                if (r == c) A[c][k] = nv[m];
                else if (fv[m] != 0.0) A[r][k] -= fv[m] * nv[m];
            }
        }
        __syncthreads();
    }
    return 1;
}

// Reductions of the CG steps (p.Kp, r.z0, r.r, C z0) go to striped FP64
// accumulators: a workgroup adds its wave sums to stripe (block index mod
// ACC_STRIPES) with hardware atomics, so no address sees more than a few dozen
// adds; the finishing kernel sums the stripes and clears them.  Record k of load
// case w of problem prob: acc_index<C>(prob, R, w, k, stripe).
constexpr int ACC_STRIPES = 32;
template <int C> constexpr int ACC_RECMAX = 2 + C * 4;
template <int C>
__host__ __device__ inline long long acc_index(int prob, int R, int w, int k, int stripe) {
    return (((long long)prob * R + w) * ACC_RECMAX<C> + k) * ACC_STRIPES + stripe;
}

// Wavefront sum of a double (64 lanes).
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Wavefront sums of N <= 16 doubles with the values spread over the lanes:
// with M = N rounded up to a power of two, each of the first log2(M) exchange
// rounds halves the values a lane carries (it keeps one half of them and
// sends the other half to its partner), and the remaining rounds finish the
// single value left.  Every entry is summed over the same pairing tree, in the
// same operand order, as the plain butterfly, so the totals are those of
// wave_sum bit for bit, with M - 1 + (6 - log2 M) exchanges instead of 6 N.
// Returns this lane's total; k receives its entry, which the lanes with
// (lane & (64 / M - 1)) == 0 hold once each (entries k >= N are padding).
template <int N>
__device__ inline double wave_sums_spread(const double *v, int &k) {
    static_assert(N >= 1 && N <= 16, "at most 16 values");
    constexpr int M = N <= 1 ? 1 : N <= 2 ? 2 : N <= 4 ? 4 : N <= 8 ? 8 : 16;
    const int lane = threadIdx.x & 63;
    double a[M];
#pragma unroll
    for (int j = 0; j < M; ++j) a[j] = j < N ? v[j] : 0.0;
    int idx = 0, off = 32;
#pragma unroll
    for (int m = M; m > 1; m >>= 1, off >>= 1) {
        const bool hi = (lane & off) != 0;
        const int half = m >> 1;
#pragma unroll
        for (int j = 0; j < half; ++j) {
            const double send = hi ? a[j] : a[j + half];
            const double keep = hi ? a[j + half] : a[j];
            a[j] = keep + __shfl_xor(send, off, 64);
        }
        idx += hi ? half : 0;
    }
    double s = a[0];
#pragma unroll
    for (; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    k = idx;
    return s;
}
// Lanes that write the totals of wave_sums_spread<N>.
template <int N>
__device__ inline bool wave_spread_writer(int lane) {
    constexpr int M = N <= 1 ? 1 : N <= 2 ? 2 : N <= 4 ? 4 : N <= 8 ? 8 : 16;
    return (lane & (64 / M - 1)) == 0;
}

}  // namespace chom
