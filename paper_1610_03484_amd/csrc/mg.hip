// Two-level preconditioner for CG on the order-p hierarchic systems.
//
// The paper factorises the RVE system directly (Sec. 2); for CG this library
// adds a coarse space to the point-block Jacobi matrix M:
//
//   B = M^-1 + Q V Q^T,   Q = P_0 P_1.
//
// P_0 injects vertex values: the vertex functions of the hierarchic basis are
// the P1 hats, so P_0^T K P_0 is the P1 stiffness matrix A_0 of the same tets
// (no triple product).  The P1 spaces of the Kuhn grids with n, n/2, n/4, ...
// cells nest -- the Kuhn split of a grid is refined by the Kuhn split of the grid
// with half the spacing, every fine vertex being a coarse vertex or the midpoint
// of a coarse Kuhn edge -- so P_l is linear interpolation and the coarse matrices
// are the Galerkin products A_{l+1} = P_l^T A_l P_l, each a 15-point stencil of
// C x C blocks.  V is one symmetric V(1,1) cycle from level 1 (the n/2 grid)
// down; the vertex grid itself is not smoothed: its l1 block Jacobi would repeat
// the point-block Jacobi of M at the vertices (whose diagonal blocks are those
// of A_0), and a V-cycle from level 0 measured the same CG step counts at
// 40% more time per step.  Smoother: l1
// block Jacobi (the diagonal block plus the absolute off-block row sums on its
// diagonal), convergent with no damping parameter; the coarsest level takes a
// fixed number of such sweeps.  V is therefore a fixed symmetric positive
// definite operator and the iteration stays preconditioned CG.
//
// Layouts, per problem from Prob.moff (points): stencils [pt][15][C*C] (slot order
// of kuhn_offset, block row-major: row = test component), l1 inverses [pt][MS]
// (packed as the point-block Jacobi inverse), vectors [R][mg_pts][C], restricted
// constraint rows of level 1 [pt][4] (FP64).  Dirichlet problems keep their
// boundary points with zero rows and inverses, so every vector is zero there.
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "internal.h"

namespace chom {

void mg_levels(Geo &G) {
    G.mg_nlev = 0;
    G.mg_pts = 0;
    if (G.n % 2 != 0 || G.n < 6) return;
    int nl = G.n, cnt = 0;
    long long off = 0;
    while (cnt < MG_MAXLEV) {
        G.mg_n[cnt] = nl;
        G.mg_lw[cnt] = (G.bc == 1) ? nl : nl + 1;
        G.mg_off[cnt] = off;
        off += (long long)G.mg_lw[cnt] * G.mg_lw[cnt] * G.mg_lw[cnt];
        ++cnt;
        if (nl % 2 != 0 || nl / 2 < 3) break;
        nl /= 2;
    }
    if (cnt < 2) return;   // the coarse space starts on level 1
    G.mg_nlev = cnt;
    G.mg_pts = off;
}

void mg_tables(const Geo &G, std::vector<int> &nbr, std::vector<int> &child, std::vector<int> &par) {
    const long long tot = G.mg_pts;
    nbr.assign((size_t)tot * 16, 0);
    child.assign((size_t)tot * 16, -1);
    par.assign((size_t)tot * 16, 0);
    const bool per = G.bc == 1, dir = G.bc == 0;
    auto wrapi = [](int i, int n) { i %= n; return i < 0 ? i + n : i; };
    auto index = [&](int l, int i, int j, int k) -> long long {   // -1 outside
        const int n = G.mg_n[l], lw = G.mg_lw[l];
        if (per) {
            i = wrapi(i, n); j = wrapi(j, n); k = wrapi(k, n);
        } else if (i < 0 || j < 0 || k < 0 || i > n || j > n || k > n) {
            return -1;
        }
        return (long long)i + (long long)lw * ((long long)j + (long long)lw * k);
    };
    auto boundary = [&](int l, int i, int j, int k) {
        const int n = G.mg_n[l];
        return dir && (i == 0 || j == 0 || k == 0 || i == n || j == n || k == n);
    };
    for (int l = 0; l < G.mg_nlev; ++l) {
        const int lw = G.mg_lw[l];
        const long long np = (long long)lw * lw * lw;
        for (long long pt = 0; pt < np; ++pt) {
            const int i = (int)(pt % lw), j = (int)((pt / lw) % lw), k = (int)(pt / ((long long)lw * lw));
            const size_t row = (size_t)(G.mg_off[l] + pt) * 16;
            for (int s = 0; s < MG_SLOTS; ++s) {
                int dx, dy, dz;
                kuhn_offset(s, dx, dy, dz);
                const long long q = index(l, i + dx, j + dy, k + dz);
                nbr[row + s] = (int)(q < 0 ? pt : q);
            }
            if (l >= 1) {
                for (int m = 0; m < MG_SLOTS; ++m) {
                    int ox, oy, oz;
                    kuhn_offset(m, ox, oy, oz);
                    int fi = 2 * i + ox, fj = 2 * j + oy, fk = 2 * k + oz;
                    const long long f = index(l - 1, fi, fj, fk);
                    if (f < 0 || boundary(l, i, j, k)) continue;
                    if (l == 1) {
                        if (boundary(0, fi, fj, fk)) continue;
                        if (per) {
                            fi = wrapi(fi, G.mg_n[0]); fj = wrapi(fj, G.mg_n[0]); fk = wrapi(fk, G.mg_n[0]);
                        }
                        const int p = G.p;
                        child[row + m] = (int)((long long)(p * fi) + (long long)G.Lw * ((long long)(p * fj) + (long long)G.Lw * (p * fk)));
                    } else {
                        child[row + m] = (int)f;
                    }
                }
            }
            if (l + 1 < G.mg_nlev) {
                const int px = i & 1, py = j & 1, pz = k & 1;
                par[row + 0] = (int)index(l + 1, (i - px) >> 1, (j - py) >> 1, (k - pz) >> 1);
                par[row + 1] = (int)index(l + 1, (i + px) >> 1, (j + py) >> 1, (k + pz) >> 1);
            }
        }
    }
}

namespace {

constexpr int MG_BS = 256;

inline int grid_cap(long long work, int bs, int cap) {
    long long g = (work + bs - 1) / bs;
    if (g < 1) g = 1;
    return (int)(g < cap ? g : cap);
}

struct Lev {
    int n, lw, per, dir;
    long long off;
};

__device__ inline Lev level_of(const Geo &G, int l) {
    Lev V;
    V.n = G.mg_n[l];
    V.lw = G.mg_lw[l];
    V.off = G.mg_off[l];
    V.per = G.bc == 1;
    V.dir = G.bc == 0;
    return V;
}

__device__ inline int wrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// Index of level point (i, j, k) (any integers for periodic levels), or -1 outside.
__device__ inline long long lev_index(const Lev &V, int i, int j, int k) {
    if (V.per) {
        i = wrap(i, V.n);
        j = wrap(j, V.n);
        k = wrap(k, V.n);
    } else if (i < 0 || j < 0 || k < 0 || i > V.n || j > V.n || k > V.n) {
        return -1;
    }
    return (long long)i + (long long)V.lw * ((long long)j + (long long)V.lw * k);
}

__device__ inline bool lev_boundary(const Lev &V, int i, int j, int k) {
    return V.dir && (i == 0 || j == 0 || k == 0 || i == V.n || j == V.n || k == V.n);
}

// Coordinates of level point pt (levels hold far fewer than 2^31 points).
__device__ inline void lev_xyz(const Lev &V, long long pt, int &i, int &j, int &k) {
    const int q = (int)pt, lw = V.lw;
    const int t = q / lw;
    i = q - t * lw;
    k = t / lw;
    j = t - k * lw;
}

// ------------------------------------------------------------------ setup (FP64)
// The tets that hold both a vertex I and its Kuhn neighbour J = I + offset(s)
// are the same for every I: tet t of the cell whose corner d (bits x, y, z) is
// I, with I and J its vertices va and vb.  Tabulated at compile time per slot
// (24 pairs for I itself, 84 over the 15 slots).
struct Asm0Table {
    int start[MG_SLOTS + 1];
    int code[MG_SLOTS * 48];   // d | t << 3 | va << 6 | vb << 8
};
constexpr Asm0Table make_asm0_table() {
    Asm0Table T{};
    constexpr int ox[8] = {0, 1, 0, 0, 1, 1, 0, 1}, oy[8] = {0, 0, 1, 0, 1, 0, 1, 1}, oz[8] = {0, 0, 0, 1, 0, 1, 1, 1};
    constexpr int pa[6] = {0, 0, 1, 1, 2, 2}, pb[6] = {1, 2, 0, 2, 0, 1};   // the Kuhn permutations
    int n = 0;
    for (int s = 0; s < MG_SLOTS; ++s) {
        T.start[s] = n;
        const int b0 = s < 8 ? s : s - 7, sg = s < 8 ? 1 : -1;
        const int dx = sg * ox[b0], dy = sg * oy[b0], dz = sg * oz[b0];
        for (int d = 0; d < 8; ++d) {
            const int ax = d & 1, ay = (d >> 1) & 1, az = (d >> 2) & 1;
            const int bx = ax + dx, by = ay + dy, bz = az + dz;
            if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;
            for (int t = 0; t < 6; ++t) {
                int va = -1, vb = -1;
                for (int q = 0; q < 4; ++q) {
                    int c3[3] = {0, 0, 0};
                    if (q >= 1) c3[pa[t]] = 1;
                    if (q >= 2) c3[pb[t]] = 1;
                    if (q == 3) c3[0] = c3[1] = c3[2] = 1;
                    if (c3[0] == ax && c3[1] == ay && c3[2] == az) va = q;
                    if (c3[0] == bx && c3[1] == by && c3[2] == bz) vb = q;
                }
                if (va < 0 || vb < 0) continue;
                T.code[n++] = d | t << 3 | va << 6 | vb << 8;
            }
        }
    }
    T.start[MG_SLOTS] = n;
    return T;
}
__constant__ Asm0Table c_asm0 = make_asm0_table();
static_assert(make_asm0_table().start[1] == 24, "every cube corner lies in the tets of the Kuhn split");

// Level 0: A_0[I][s] = sum over tets holding I and J = I + offset(s) of
// |e| (grad lam_J . C . grad lam_I) (mechanics: the C x C block with
// entry [c][d] = |e| sum_j sigma(sym(e_d x g_J))[c][j] g_I[j]).
template <int C>
__global__ void mg_assemble0_kernel(const Geo *geos, const Prob *probs, double *A64) {
    constexpr int CC = C * C;
    const Prob &P = probs[blockIdx.y];
    const Geo &G = geos[P.geo];
    if (G.mg_nlev == 0) return;
    const Lev V = level_of(G, 0);
    const int n = G.n;
    const long long np = (long long)V.lw * V.lw * V.lw;
    double *Ap = A64 + (P.moff + V.off) * MG_SLOTS * CC;
    for (long long u = blockIdx.x * (long long)blockDim.x + threadIdx.x; u < np * MG_SLOTS;
         u += (long long)gridDim.x * blockDim.x) {
        // slot-major: the threads of a wave share a slot (and so the table's loop)
        const int s = (int)(u / np);
        const long long pt = u - (long long)s * np;
        int i, j, k, dx, dy, dz;
        lev_xyz(V, pt, i, j, k);
        kuhn_offset(s, dx, dy, dz);
        double acc[CC];
#pragma unroll
        for (int q = 0; q < CC; ++q) acc[q] = 0.0;
        const bool inside = V.per || (i + dx >= 0 && j + dy >= 0 && k + dz >= 0 && i + dx <= n && j + dy <= n && k + dz <= n);
        if (inside && !lev_boundary(V, i, j, k) && !lev_boundary(V, i + dx, j + dy, k + dz)) {
            for (int e = c_asm0.start[s]; e < c_asm0.start[s + 1]; ++e) {
                const int code = c_asm0.code[e];
                const int d = code & 7, t = (code >> 3) & 7, va = (code >> 6) & 3, vb = (code >> 8) & 3;
                const int ax = d & 1, ay = (d >> 1) & 1, az = (d >> 2) & 1;   // I's corner in the cell
                int cx = i - ax, cy = j - ay, cz = k - az;
                if (V.per) {
                    cx = wrap(cx, n);
                    cy = wrap(cy, n);
                    cz = wrap(cz, n);
                } else if (cx < 0 || cy < 0 || cz < 0 || cx >= n || cy >= n || cz >= n) {
                    continue;
                }
                {
                    const long long tet = ((long long)cx + (long long)n * ((long long)cy + (long long)n * cz)) * 6 + t;
                    double g[4][3], vol, a[3];
                    int ph;
                    GeoSel<double>::get(G, tet, t, g, vol);
                    GeoSel<double>::elem(G, tet, a, ph);
                    const double *m = P.mat64[ph ? 1 : 0];
                    if constexpr (C == 3) {
                        for (int dd = 0; dd < 3; ++dd) {
                            double Gm[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
                            for (int l2 = 0; l2 < 3; ++l2) Gm[dd][l2] = g[vb][l2];
                            const double e[6] = {Gm[0][0], Gm[1][1], Gm[2][2], 0.5 * (Gm[0][1] + Gm[1][0]),
                                                 0.5 * (Gm[1][2] + Gm[2][1]), 0.5 * (Gm[2][0] + Gm[0][2])};
                            double sg[6];
                            stress_ti<double>(e, a, m, sg);
                            const double *ga = g[va];
                            acc[0 * 3 + dd] += vol * (sg[0] * ga[0] + sg[3] * ga[1] + sg[5] * ga[2]);
                            acc[1 * 3 + dd] += vol * (sg[3] * ga[0] + sg[1] * ga[1] + sg[4] * ga[2]);
                            acc[2 * 3 + dd] += vol * (sg[5] * ga[0] + sg[4] * ga[1] + sg[2] * ga[2]);
                        }
                    } else {
                        double fl[3];
                        flux_ti<double>(g[vb], a, m, fl);
                        acc[0] += vol * (fl[0] * g[va][0] + fl[1] * g[va][1] + fl[2] * g[va][2]);
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < CC; ++q) Ap[(pt * MG_SLOTS + s) * CC + q] = acc[q];
    }
}

// Galerkin product on nested Kuhn grids in relative form: the fine children of
// a coarse point sit at 2 I + o_m (the 15 stencil offsets o_m, weight 1 for the
// point itself, 1/2 for an edge midpoint) and a fine neighbour 2 I + o_m + o_q
// prolongs from its even parent(s); which (m, q) pairs reach coarse slot s, and
// with which weight, does not depend on I.  The pairs (421 over the 15 slots)
// are tabulated at compile time.
struct RapTable {
    int start[MG_SLOTS + 1];
    int code[448];   // m | q << 4 | wcode << 8 (weight 1, 1/2, 1/4 for wcode 0, 1, 2)
};
constexpr int rap_off(int k, int d) {
    constexpr int ox[8] = {0, 1, 0, 0, 1, 1, 0, 1}, oy[8] = {0, 0, 1, 0, 1, 0, 1, 1}, oz[8] = {0, 0, 0, 1, 0, 1, 1, 1};
    const int b = k < 8 ? k : k - 7, sg = k < 8 ? 1 : -1;
    return sg * (d == 0 ? ox[b] : d == 1 ? oy[b] : oz[b]);
}
constexpr int rap_half(int v) { return v >= 0 ? v / 2 : -((-v + 1) / 2); }   // floor(v / 2)
constexpr RapTable make_rap_table() {
    RapTable t{};
    int n = 0;
    for (int s = 0; s < MG_SLOTS; ++s) {
        t.start[s] = n;
        for (int m = 0; m < MG_SLOTS; ++m)
            for (int q = 0; q < MG_SLOTS; ++q) {
                int g[3] = {0, 0, 0}, par[3] = {0, 0, 0}, d[3] = {0, 0, 0};
                bool even = true;
                for (int a = 0; a < 3; ++a) {
                    g[a] = rap_off(m, a) + rap_off(q, a);
                    par[a] = g[a] & 1;
                    d[a] = rap_off(s, a);
                    if (par[a]) even = false;
                }
                int w2 = 0;   // wj in halves
                if (even) {
                    bool hit = true;
                    for (int a = 0; a < 3; ++a) hit = hit && rap_half(g[a]) == d[a];
                    if (hit) w2 = 2;
                } else {
                    bool lo = true, hi = true;
                    for (int a = 0; a < 3; ++a) {
                        lo = lo && rap_half(g[a] - par[a]) == d[a];
                        hi = hi && rap_half(g[a] + par[a]) == d[a];
                    }
                    w2 = (lo ? 1 : 0) + (hi ? 1 : 0);
                }
                if (w2 == 0) continue;
                // w = wi * wj, wi = 1 (m = 0) or 1/2; wj = w2 / 2
                const int wcode = (m == 0 ? 0 : 1) + (w2 == 2 ? 0 : 1);
                t.code[n++] = m | (q << 4) | (wcode << 8);
            }
    }
    t.start[MG_SLOTS] = n;
    return t;
}
__constant__ RapTable c_rap = make_rap_table();
static_assert(make_rap_table().start[MG_SLOTS] == 421, "Galerkin pair count of the 15-point Kuhn stencil");

// Level l + 1 from level l: A_c[I][s] = sum_{i child of I} sum_{j fine neighbour
// of i, J parent of j, J = I + offset(s)} w_iI A_f[i][j] w_jJ.  Coordinates stay
// unwrapped (geometric) until a level array is indexed, so a coupling is credited
// to the slot of its geometric offset.
// Work item (slot, coarse point), slot-major so a wave walks one slot's pairs;
// every pair's block is loaded unconditionally (an absent or boundary child
// weighs 0 and reads the point's own block), so the loads of consecutive pairs
// are in flight together.
template <int C>
__global__ void mg_rap_kernel(const Geo *geos, const Prob *probs, int l, double *A64) {
    constexpr int CC = C * C;
    const Prob &P = probs[blockIdx.y];
    const Geo &G = geos[P.geo];
    if (G.mg_nlev <= l + 1) return;
    const Lev F = level_of(G, l), Cv = level_of(G, l + 1);
    const long long npc = (long long)Cv.lw * Cv.lw * Cv.lw;
    const double *Af = A64 + (P.moff + F.off) * MG_SLOTS * CC;
    double *Ac = A64 + (P.moff + Cv.off) * MG_SLOTS * CC;
    for (long long u = blockIdx.x * (long long)blockDim.x + threadIdx.x; u < npc * MG_SLOTS;
         u += (long long)gridDim.x * blockDim.x) {
        const int s = (int)(u / npc);
        const long long pt = u - s * npc;
        int I, Jy, K, dx, dy, dz;
        lev_xyz(Cv, pt, I, Jy, K);
        kuhn_offset(s, dx, dy, dz);
        const int TX = I + dx, TY = Jy + dy, TZ = K + dz;   // target coarse point (unwrapped)
        double acc[CC];
#pragma unroll
        for (int q = 0; q < CC; ++q) acc[q] = 0.0;
        const bool ok = lev_index(Cv, TX, TY, TZ) >= 0 && !lev_boundary(Cv, I, Jy, K) &&
                        !lev_boundary(Cv, TX, TY, TZ);
        if (ok) {
            const int e1 = c_rap.start[s + 1];
#pragma unroll 4
            for (int e = c_rap.start[s]; e < e1; ++e) {
                const int code = c_rap.code[e];
                const int m = code & 15, q = (code >> 4) & 15, wc = code >> 8;
                int ox, oy, oz;
                kuhn_offset(m, ox, oy, oz);
                const int fi = 2 * I + ox, fj = 2 * Jy + oy, fk = 2 * K + oz;   // child (unwrapped)
                const long long f0 = lev_index(F, fi, fj, fk);
                const bool live = f0 >= 0 && !lev_boundary(F, fi, fj, fk);
                const double w = live ? (wc == 0 ? 1.0 : wc == 1 ? 0.5 : 0.25) : 0.0;
                const double *blk = Af + ((live ? f0 : 0) * MG_SLOTS + q) * CC;
#pragma unroll
                for (int c = 0; c < CC; ++c) acc[c] += w * blk[c];
            }
        }
#pragma unroll
        for (int c = 0; c < CC; ++c) Ac[(pt * MG_SLOTS + s) * CC + c] = acc[c];
    }
}

// l1 block-Jacobi inverse of every coarse point of the class, and the T copies.
template <int C>
__global__ __launch_bounds__(MG_BS) void mg_dinv_kernel(long long total, const double *A64, double *D64) {
    constexpr int CC = C * C;
    constexpr int MS = (C == 3) ? 6 : 1;
    for (long long pt = blockIdx.x * (long long)blockDim.x + threadIdx.x; pt < total;
         pt += (long long)gridDim.x * blockDim.x) {
        const double *row = A64 + pt * MG_SLOTS * CC;
        double D[CC];
#pragma unroll
        for (int e = 0; e < CC; ++e) D[e] = row[e];
        for (int s = 1; s < MG_SLOTS; ++s)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                double a = 0.0;
#pragma unroll
                for (int d = 0; d < C; ++d) a += fabs(row[s * CC + c * C + d]);
                D[c * C + c] += a;
            }
        double out[MS];
        if constexpr (C == 3) {
            const double a = D[0], b = D[4], c = D[8];
            const double xy = 0.5 * (D[1] + D[3]), yz = 0.5 * (D[5] + D[7]), xz = 0.5 * (D[2] + D[6]);
            const double c00 = b * c - yz * yz, c11 = a * c - xz * xz, c22 = a * b - xy * xy;
            const double c01 = xz * yz - xy * c, c12 = xy * xz - a * yz, c02 = xy * yz - b * xz;
            const double det = a * c00 + xy * c01 + xz * c02;
            const double id = det > 0.0 ? 1.0 / det : 0.0;
            out[0] = c00 * id;
            out[1] = c11 * id;
            out[2] = c22 * id;
            out[3] = c01 * id;
            out[4] = c12 * id;
            out[5] = c02 * id;
        } else {
            out[0] = D[0] > 0.0 ? 1.0 / D[0] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < MS; ++e) D64[pt * MS + e] = out[e];
    }
}

__global__ void mg_to_float_kernel(long long n, const double *src, float *dst) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

// Level-1 restricted constraint rows: rows1[I][k] = sum over the level-0 children
// v of I (weights 1 and 1/2) of the fine row k at vertex v (FP64, all 4 rows).
__global__ void mg_rows1_kernel(const Geo *geos, const Prob *probs, double *rows1) {
    const Prob &P = probs[blockIdx.y];
    const Geo &G = geos[P.geo];
    if (G.mg_nlev == 0) return;
    const Lev F = level_of(G, 0), Cv = level_of(G, 1);
    const long long np = (long long)Cv.lw * Cv.lw * Cv.lw;
    const int p = G.p;
    for (long long pt = blockIdx.x * (long long)blockDim.x + threadIdx.x; pt < np; pt += (long long)gridDim.x * blockDim.x) {
        int I, J, K;
        lev_xyz(Cv, pt, I, J, K);
        double acc[4] = {0, 0, 0, 0};
        for (int m = 0; m < MG_SLOTS; ++m) {
            int ox, oy, oz;
            kuhn_offset(m, ox, oy, oz);
            int fi = 2 * I + ox, fj = 2 * J + oy, fk = 2 * K + oz;
            if (lev_index(F, fi, fj, fk) < 0) continue;
            if (F.per) {
                fi = wrap(fi, F.n);
                fj = wrap(fj, F.n);
                fk = wrap(fk, F.n);
            }
            const long long lat = (long long)(p * fi) + (long long)G.Lw * ((long long)(p * fj) + (long long)G.Lw * (p * fk));
            const double wgt = (m == 0) ? 1.0 : 0.5;
            for (int k = 0; k < 4; ++k) acc[k] += wgt * G.rows[4 * lat + k];
        }
        for (int k = 0; k < 4; ++k) rows1[(P.moff + Cv.off + pt) * 4 + k] = acc[k];
    }
}

// ------------------------------------------------------------------ V-cycle
// The coarse correction starts on level 1 (the n/2 grid): its right side is
// r_1 = P_1^T P^T r, gathered from the fine vector at the vertex lattice points.
// Per (problem, load case) and level l the vectors are r (restricted right
// side), xp = D^-1 r (the pre-smoothed iterate from zero), res (r - A xp; later
// the corrected iterate xc = xp + P e_{l+1}) and x (the level's output e_l).
// Level 1 runs over the whole grid; levels 2 .. coarsest of one (problem, load
// case) run in one workgroup (mg_fused_kernel), in LDS when they fit.

template <typename T>
struct LV {   // vectors of one level for one (problem, load case), each [points][C]
    T *r, *xp, *res, *x;
};

template <typename T, int C, int R>
__device__ inline LV<T> level_vecs(const Geo &G, const Prob &P, int w, const Lev &V, T *r, T *xp, T *res, T *x) {
    const long long o = (P.moff * R + (long long)w * G.mg_pts + V.off) * C;
    return LV<T>{r + o, xp + o, res + o, x + o};
}

template <typename T, int C>
__device__ inline void load_c(const T *p, T v[C]) {
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = p[c];
}

template <typename T, int C>
__device__ inline void store_c(T *p, const T v[C]) {
#pragma unroll
    for (int c = 0; c < C; ++c) p[c] = v[c];
}

// acc -= sum_s A[s] v[nb[s]] (A: the point's 15 blocks; nb: its row of the
// neighbour table -- outside the lattice the point itself, whose block is zero).
template <typename T, int C>
__device__ inline void apply_stencil(const int *nb, const T *Arow, const T *v, T acc[C]) {
    constexpr int CC = C * C;
#pragma unroll
    for (int s = 0; s < MG_SLOTS; ++s) {
        T vq[C];
        load_c<T, C>(v + (long long)nb[s] * C, vq);
        const T *blk = Arow + s * CC;
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int d = 0; d < C; ++d) acc[c] -= blk[c * C + d] * vq[d];
    }
}

__device__ inline const int *row16(const int *table, const Lev &V, long long pt) {
    return table + (V.off + pt) * 16;
}

// res = r - A xp.
template <typename T, int C>
__device__ inline void resid_pt(const Geo &G, const Lev &V, const T *A, LV<T> v, long long pt) {
    constexpr int CC = C * C;
    T acc[C];
    load_c<T, C>(v.r + pt * C, acc);
    apply_stencil<T, C>(row16(G.mg_nbr, V, pt), A + pt * MG_SLOTS * CC, v.xp, acc);
    store_c<T, C>(v.res + pt * C, acc);
}

// r_{l+1}[I] = sum of the children of I (I with weight 1, the midpoints of its
// 14 Kuhn edges with weight 1/2) of res_l; xp_{l+1} = D^-1 r_{l+1}.
template <typename T, int C>
__device__ inline void restrict_pt(const Geo &G, const Lev &Cv, const T *Dinv, LV<T> vf, LV<T> vc, long long pt) {
    constexpr int MS = (C == 3) ? 6 : 1;
    const int *ch = row16(G.mg_child, Cv, pt);
    T acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = T(0);
#pragma unroll
    for (int m = 0; m < MG_SLOTS; ++m) {
        const int f = ch[m];
        const T wgt = f < 0 ? T(0) : (m == 0 ? T(1) : T(0.5));
        const long long fs = f < 0 ? 0 : f;
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] += wgt * vf.res[fs * C + c];
    }
    store_c<T, C>(vc.r + pt * C, acc);
    T xv[C];
    minv_apply<T, C>(Dinv + pt * MS, acc, xv);
    store_c<T, C>(vc.xp + pt * C, xv);
}

// Prolongation of the level-(l+1) vector e to level-l point pt: the mean of e at
// its two parents (equal for a point with even coordinates).
template <typename T, int C>
__device__ inline void prolong(const Geo &G, const Lev &V, const T *e, long long pt, T out[C]) {
    const int *pa = row16(G.mg_par, V, pt);
    const long long a = pa[0], b = pa[1];
#pragma unroll
    for (int c = 0; c < C; ++c) out[c] = T(0.5) * (e[a * C + c] + e[b * C + c]);
}

// xc = xp + P e_{l+1}, stored in res (e vanishes at Dirichlet boundary points).
template <typename T, int C>
__device__ inline void correct_pt(const Geo &G, const Lev &V, LV<T> v, const T *e, long long pt) {
    T xv[C], pe[C];
    load_c<T, C>(v.xp + pt * C, xv);
    prolong<T, C>(G, V, e, pt, pe);
#pragma unroll
    for (int c = 0; c < C; ++c) xv[c] += pe[c];
    store_c<T, C>(v.res + pt * C, xv);
}

// x = xc + D^-1 (r - A xc).
template <typename T, int C>
__device__ inline void post_pt(const Geo &G, const Lev &V, const T *A, const T *Dinv, LV<T> v, long long pt) {
    constexpr int CC = C * C;
    constexpr int MS = (C == 3) ? 6 : 1;
    T acc[C];
    load_c<T, C>(v.r + pt * C, acc);
    apply_stencil<T, C>(row16(G.mg_nbr, V, pt), A + pt * MG_SLOTS * CC, v.res, acc);
    T d[C], xi[C];
    minv_apply<T, C>(Dinv + pt * MS, acc, d);
    load_c<T, C>(v.res + pt * C, xi);
#pragma unroll
    for (int c = 0; c < C; ++c) xi[c] += d[c];
    store_c<T, C>(v.x + pt * C, xi);
}

template <typename T, int C, int R>
struct VPtr {
    const T *fine_r;
    const T *A, *Dinv;
    T *r, *xp, *res, *x;
    const double *rows1;
};

#define MG_LEVEL_KERNEL_HEAD(LEVEL_OK)                                            \
    const int prob = blockIdx.y;                                                  \
    if (prob_active != nullptr && prob_active[prob] == 0) return;                 \
    const Prob &P = probs[prob];                                                  \
    const Geo &G = geos[P.geo];                                                   \
    if (!(LEVEL_OK)) return;                                                      \
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;

// The level-1 kernels: wave g takes load cases KG g .. KG g + KG - 1 of a
// problem, so a point's index tables, stencil blocks, inverse block and
// constraint rows are read once for all of them.
template <typename T, int C, int R, int KG>
__device__ inline void level_vecs_kg(const Geo &G, const Prob &P, int c0, const Lev &V, const VPtr<T, C, R> &Q,
                                     LV<T> (&v)[KG]) {
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) v[kk] = level_vecs<T, C, R>(G, P, c0 + kk, V, Q.r, Q.xp, Q.res, Q.x);
}

// acc[kk] -= sum_s A[s] v[kk][nb[s]] for the KG vectors (each block loaded once).
template <typename T, int C, int KG>
__device__ inline void apply_stencil_kg(const int *nb, const T *Arow, const T *const (&v)[KG], T (&acc)[KG][C]) {
    constexpr int CC = C * C;
#pragma unroll
    for (int s = 0; s < MG_SLOTS; ++s) {
        const long long j = nb[s];
        T blk[CC];
#pragma unroll
        for (int e = 0; e < CC; ++e) blk[e] = Arow[s * CC + e];
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
            T vq[C];
            load_c<T, C>(v[kk] + j * C, vq);
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int d = 0; d < C; ++d) acc[kk][c] -= blk[c * C + d] * vq[d];
        }
    }
}

// r_1[I] = sum over the level-0 children v of I of the fine right side at v
// (children on a Dirichlet boundary and outside the lattice are absent from the
// table); xp_1 = D^-1 r_1.
template <typename T, int C, int R, int KG>
__global__ __launch_bounds__(64 * (R / KG)) void mg_restrict01_kernel(const Geo *geos, const Prob *probs,
                                                                      VPtr<T, C, R> Q, const int *prob_active) {
    constexpr int MS = (C == 3) ? 6 : 1;
    MG_LEVEL_KERNEL_HEAD(G.mg_nlev >= 2)
    const int c0 = w * KG;
    const Lev V = level_of(G, 1);
    LV<T> v[KG];
    level_vecs_kg<T, C, R, KG>(G, P, c0, V, Q, v);
    const T *D = Q.Dinv + (P.moff + V.off) * MS;
    const long long np = (long long)V.lw * V.lw * V.lw;
    for (long long pt = blockIdx.x * 64LL + lane; pt < np; pt += gridDim.x * 64LL) {
        const int *ch = row16(G.mg_child, V, pt);
        int f[MG_SLOTS];
#pragma unroll
        for (int m = 0; m < MG_SLOTS; ++m) f[m] = ch[m];
        T Mi[MS];
#pragma unroll
        for (int k = 0; k < MS; ++k) Mi[k] = D[pt * MS + k];
        T acc[KG][C];
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
            const T *fr = Q.fine_r + P.voff + (long long)(c0 + kk) * G.npts * C;
#pragma unroll
            for (int c = 0; c < C; ++c) acc[kk][c] = T(0);
#pragma unroll
            for (int m = 0; m < MG_SLOTS; ++m) {
                T vv[C];
                load_c<T, C>(fr + (long long)(f[m] < 0 ? 0 : f[m]) * C, vv);
                const T wgt = f[m] < 0 ? T(0) : (m == 0 ? T(1) : T(0.5));
#pragma unroll
                for (int c = 0; c < C; ++c) acc[kk][c] += wgt * vv[c];
            }
        }
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
            store_c<T, C>(v[kk].r + pt * C, acc[kk]);
            T xv[C];
            minv_apply<T, C>(Mi, acc[kk], xv);
            store_c<T, C>(v[kk].xp + pt * C, xv);
        }
    }
}

// res = r - A xp on level 1.
template <typename T, int C, int R, int KG>
__global__ __launch_bounds__(64 * (R / KG)) void mg_resid1_kernel(const Geo *geos, const Prob *probs,
                                                                  VPtr<T, C, R> Q, const int *prob_active) {
    constexpr int CC = C * C;
    MG_LEVEL_KERNEL_HEAD(G.mg_nlev >= 3)
    const int c0 = w * KG;
    const Lev V = level_of(G, 1);
    LV<T> v[KG];
    level_vecs_kg<T, C, R, KG>(G, P, c0, V, Q, v);
    const T *xps[KG];
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) xps[kk] = v[kk].xp;
    const T *A = Q.A + (P.moff + V.off) * MG_SLOTS * CC;
    const long long np = (long long)V.lw * V.lw * V.lw;
    for (long long pt = blockIdx.x * 64LL + lane; pt < np; pt += gridDim.x * 64LL) {
        T acc[KG][C];
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) load_c<T, C>(v[kk].r + pt * C, acc[kk]);
        apply_stencil_kg<T, C, KG>(row16(G.mg_nbr, V, pt), A + pt * MG_SLOTS * CC, xps, acc);
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) store_c<T, C>(v[kk].res + pt * C, acc[kk]);
    }
}

// xc = xp + P e_2 on level 1, stored in res.
template <typename T, int C, int R, int KG>
__global__ __launch_bounds__(64 * (R / KG)) void mg_correct1_kernel(const Geo *geos, const Prob *probs,
                                                                    VPtr<T, C, R> Q, const int *prob_active) {
    MG_LEVEL_KERNEL_HEAD(G.mg_nlev >= 3)
    const int c0 = w * KG;
    const Lev V = level_of(G, 1), Cv = level_of(G, 2);
    LV<T> v[KG], vc[KG];
    level_vecs_kg<T, C, R, KG>(G, P, c0, V, Q, v);
    level_vecs_kg<T, C, R, KG>(G, P, c0, Cv, Q, vc);
    const long long np = (long long)V.lw * V.lw * V.lw;
    for (long long pt = blockIdx.x * 64LL + lane; pt < np; pt += gridDim.x * 64LL) {
        const int *pa = row16(G.mg_par, V, pt);
        const long long ia = pa[0], ib = pa[1];
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
            T xv[C];
            load_c<T, C>(v[kk].xp + pt * C, xv);
            const T *e = vc[kk].x;
#pragma unroll
            for (int c = 0; c < C; ++c) xv[c] += T(0.5) * (e[ia * C + c] + e[ib * C + c]);
            store_c<T, C>(v[kk].res + pt * C, xv);
        }
    }
}

// Level-1 post-smoothing x = xc + D^-1 (r - A xc); with `accbuf`, the sums
// r_1 . e_1 (= r . Q e_1) and rows1 . e_1 (= C Q e_1) are added to the CG
// step's striped accumulators.
template <typename T, int C, int R, int NR, int KG>
__global__ __launch_bounds__(64 * (R / KG)) void mg_post1_kernel(const Geo *geos, const Prob *probs,
                                                                 VPtr<T, C, R> Q, double *accbuf,
                                                                 const int *prob_active) {
    constexpr int CC = C * C;
    constexpr int MS = (C == 3) ? 6 : 1;
    constexpr int REC = 2 + C * NR;
    const int prob = blockIdx.y;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c0 = w * KG;
    double pacc[KG][REC];
#pragma unroll
    for (int kk = 0; kk < KG; ++kk)
#pragma unroll
        for (int k = 0; k < REC; ++k) pacc[kk][k] = 0.0;
    const Prob &P = probs[prob];
    const Geo &G = geos[P.geo];
    if ((prob_active == nullptr || prob_active[prob] != 0) && G.mg_nlev >= 2) {
        const bool smooth = G.mg_nlev >= 3;   // level 1 coarsest: its output is final
        const Lev V = level_of(G, 1);
        LV<T> v[KG];
        level_vecs_kg<T, C, R, KG>(G, P, c0, V, Q, v);
        const T *xcs[KG];
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) xcs[kk] = v[kk].res;
        const T *A = Q.A + (P.moff + V.off) * MG_SLOTS * CC;
        const T *D = Q.Dinv + (P.moff + V.off) * MS;
        const double *r1 = Q.rows1 + (P.moff + V.off) * 4;
        const int rf = row_first(G.nrow);
        const int nr = G.nrow < NR ? G.nrow : NR;
        const long long np = (long long)V.lw * V.lw * V.lw;
        for (long long pt = blockIdx.x * 64LL + lane; pt < np; pt += gridDim.x * 64LL) {
            T rv[KG][C], ov[KG][C];
#pragma unroll
            for (int kk = 0; kk < KG; ++kk) load_c<T, C>(v[kk].r + pt * C, rv[kk]);
            if (smooth) {
                T acc[KG][C];
#pragma unroll
                for (int kk = 0; kk < KG; ++kk)
#pragma unroll
                    for (int c = 0; c < C; ++c) acc[kk][c] = rv[kk][c];
                apply_stencil_kg<T, C, KG>(row16(G.mg_nbr, V, pt), A + pt * MG_SLOTS * CC, xcs, acc);
                T Mi[MS];
#pragma unroll
                for (int k = 0; k < MS; ++k) Mi[k] = D[pt * MS + k];
#pragma unroll
                for (int kk = 0; kk < KG; ++kk) {
                    T d[C], xi[C];
                    minv_apply<T, C>(Mi, acc[kk], d);
                    load_c<T, C>(v[kk].res + pt * C, xi);
#pragma unroll
                    for (int c = 0; c < C; ++c) ov[kk][c] = xi[c] + d[c];
                    store_c<T, C>(v[kk].x + pt * C, ov[kk]);
                }
            } else {
#pragma unroll
                for (int kk = 0; kk < KG; ++kk) load_c<T, C>(v[kk].x + pt * C, ov[kk]);
            }
            if (accbuf != nullptr) {
                double row[4] = {0, 0, 0, 0};
                for (int a = 0; a < nr; ++a) row[a] = r1[pt * 4 + rf + a];
#pragma unroll
                for (int kk = 0; kk < KG; ++kk)
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        pacc[kk][0] += (double)rv[kk][c] * (double)ov[kk][c];
#pragma unroll
                        for (int a = 0; a < NR; ++a) pacc[kk][2 + c * NR + a] += row[a] * (double)ov[kk][c];
                    }
            }
        }
    }
    if (accbuf != nullptr) {
        const int stripe = blockIdx.x & (ACC_STRIPES - 1);
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
            int k;
            const double sum = wave_sums_spread<REC>(pacc[kk], k);
            if (wave_spread_writer<REC>(lane) && k < REC && k != 1)
                unsafeAtomicAdd(&accbuf[acc_index<C>(prob, R, c0 + kk, k, stripe)], sum);
        }
    }
}

// f = e_1 - W y per (problem, load case) on the n/2 grid (y: projection
// coefficients of the current CG step), into the level-1 res block.
template <typename T, int C, int R, int NR, int KG>
__global__ __launch_bounds__(64 * (R / KG)) void mg_fcorr_kernel(const Geo *geos, const Prob *probs,
                                                                 VPtr<T, C, R> Q, const T *W, const double *ycoef,
                                                                 const int *prob_active) {
    MG_LEVEL_KERNEL_HEAD(G.mg_nlev >= 2)
    const int c0 = w * KG;
    const Lev V = level_of(G, 1);
    LV<T> v[KG];
    level_vecs_kg<T, C, R, KG>(G, P, c0, V, Q, v);
    const int nr = G.nrow < NR ? G.nrow : NR;
    double yv[KG][C * NR > 0 ? C * NR : 1];
#pragma unroll
    for (int kk = 0; kk < KG; ++kk)
#pragma unroll
        for (int k = 0; k < C * NR; ++k) yv[kk][k] = ycoef[((long long)prob * R + c0 + kk) * C * NR + k];
    const long long np = (long long)V.lw * V.lw * V.lw;
    for (long long pt = blockIdx.x * 64LL + lane; pt < np; pt += gridDim.x * 64LL) {
        double f[KG][C];
#pragma unroll
        for (int kk = 0; kk < KG; ++kk)
#pragma unroll
            for (int c = 0; c < C; ++c) f[kk][c] = (double)v[kk].x[pt * C + c];
        if constexpr (NR > 0) {
            const T *Wp = W + (P.moff + V.off + pt) * (4 * C) * C;
#pragma unroll
            for (int i = 0; i < C; ++i)
#pragma unroll
                for (int a = 0; a < NR; ++a) {
                    if (a >= nr) continue;
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        const double wv = (double)Wp[(i * 4 + a) * C + c];
#pragma unroll
                        for (int kk = 0; kk < KG; ++kk) f[kk][c] -= yv[kk][i * NR + a] * wv;
                    }
                }
        }
#pragma unroll
        for (int kk = 0; kk < KG; ++kk)
#pragma unroll
            for (int c = 0; c < C; ++c) v[kk].res[pt * C + c] = (T)f[kk][c];
    }
}

constexpr int MG_FUSED_BS = 512;

// Levels 2 .. coarsest of one (load case, problem): restrict from level 1, the
// residuals, `sweeps` l1 block-Jacobi sweeps on the coarsest level, correct and
// post-smooth back up to level 2, whose output goes to global memory for level 1.
// With `lds` the vectors of levels >= 2 live in LDS (layout [level][r|xp|res|x]
// [points][C]); with `lds_sten` the coarsest stencils too.  Stages are separated
// by workgroup barriers.
template <typename T, int C, int R>
__global__ __launch_bounds__(MG_FUSED_BS) void mg_fused_kernel(const Geo *geos, const Prob *probs, VPtr<T, C, R> Q,
                                                               int sweeps, int lds, int lds_sten,
                                                               const int *prob_active) {
    constexpr int CC = C * C;
    constexpr int MS = (C == 3) ? 6 : 1;
    extern __shared__ unsigned char mg_smem[];
    const int prob = blockIdx.y, w = blockIdx.x;
    if (prob_active != nullptr && prob_active[prob] == 0) return;
    const Prob &P = probs[prob];
    const Geo &G = geos[P.geo];
    if (G.mg_nlev < 2) return;
    if (P.mg_sweeps > 0) sweeps = P.mg_sweeps;
    const int lc = G.mg_nlev - 1;   // 1: the n/2 grid itself is the coarsest
    const int tid = threadIdx.x, nt = blockDim.x;
    T *smem = (T *)mg_smem;
    // vectors of level l: levels >= 2 in LDS (when `lds`), packed in level order
    auto lvec = [&](int l) -> LV<T> {
        const Lev V = level_of(G, l);
        if (l >= 2 && lds && lc >= 2) {
            const long long np = (long long)V.lw * V.lw * V.lw * C;
            T *b = smem + 4LL * C * (V.off - G.mg_off[2]);
            return LV<T>{b, b + np, b + 2 * np, b + 3 * np};
        }
        return level_vecs<T, C, R>(G, P, w, V, Q.r, Q.xp, Q.res, Q.x);
    };
    const long long used = (lds && lc >= 2) ? 4LL * C * (G.mg_pts - G.mg_off[2]) : 0;
    // down
    for (int l = 1; l < lc; ++l) {
        const Lev F = level_of(G, l), Cv = level_of(G, l + 1);
        const long long npc = (long long)Cv.lw * Cv.lw * Cv.lw;
        const T *D = Q.Dinv + (P.moff + Cv.off) * MS;
        const LV<T> vf = lvec(l), vc = lvec(l + 1);
        for (long long pt = tid; pt < npc; pt += nt) restrict_pt<T, C>(G, Cv, D, vf, vc, pt);
        __syncthreads();
        if (l + 1 < lc) {
            const T *A = Q.A + (P.moff + Cv.off) * MG_SLOTS * CC;
            for (long long pt = tid; pt < npc; pt += nt) resid_pt<T, C>(G, Cv, A, vc, pt);
            __syncthreads();
        }
    }
    // coarsest: x <- x + D^-1 (r - A x) from x = xp, iterates alternating between x and res
    {
        const Lev V = level_of(G, lc);
        const long long np = (long long)V.lw * V.lw * V.lw;
        const T *A = Q.A + (P.moff + V.off) * MG_SLOTS * CC;
        const T *D = Q.Dinv + (P.moff + V.off) * MS;
        if (lds_sten) {
            T *sA = smem + used;
            for (long long e = tid; e < np * MG_SLOTS * CC; e += nt) sA[e] = A[e];
            A = sA;
        }
        const LV<T> v = lvec(lc);
        for (long long pt = tid; pt < np; pt += nt)
#pragma unroll
            for (int c = 0; c < C; ++c) v.x[pt * C + c] = v.xp[pt * C + c];
        __syncthreads();
        T *const b0 = v.x, *const b1 = v.res;   // iterates alternate (selected, not indexed)
        int cur = 0;
        if (np <= nt) {
            // one point per thread: neighbour indices, right side and inverse held in registers
            const bool have = tid < np;
            const long long pt = have ? tid : 0;
            int qi[MG_SLOTS];
            const int *nb = row16(G.mg_nbr, V, pt);
#pragma unroll
            for (int s2 = 0; s2 < MG_SLOTS; ++s2) qi[s2] = nb[s2];
            T rv[C], Dv[MS];
            load_c<T, C>(v.r + pt * C, rv);
#pragma unroll
            for (int e = 0; e < MS; ++e) Dv[e] = D[pt * MS + e];
            const T *Ap = A + pt * MG_SLOTS * CC;
            for (int it = 1; it < sweeps; ++it) {
                const T *xs = cur ? b1 : b0;
                T *xd = cur ? b0 : b1;
                if (have) {
                    T acc[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) acc[c] = rv[c];
#pragma unroll
                    for (int s2 = 0; s2 < MG_SLOTS; ++s2) {
                        T vq[C];
                        load_c<T, C>(xs + (long long)qi[s2] * C, vq);
                        const T *blk = Ap + s2 * CC;
#pragma unroll
                        for (int c = 0; c < C; ++c)
#pragma unroll
                            for (int d = 0; d < C; ++d) acc[c] -= blk[c * C + d] * vq[d];
                    }
                    T d[C];
                    minv_apply<T, C>(Dv, acc, d);
#pragma unroll
                    for (int c = 0; c < C; ++c) xd[pt * C + c] = xs[pt * C + c] + d[c];
                }
                __syncthreads();
                cur ^= 1;
            }
        } else {
            for (int it = 1; it < sweeps; ++it) {
                const T *xs = cur ? b1 : b0;
                T *xd = cur ? b0 : b1;
                for (long long pt = tid; pt < np; pt += nt) {
                    T acc[C];
                    load_c<T, C>(v.r + pt * C, acc);
                    apply_stencil<T, C>(row16(G.mg_nbr, V, pt), A + pt * MG_SLOTS * CC, xs, acc);
                    T d[C];
                    minv_apply<T, C>(D + pt * MS, acc, d);
#pragma unroll
                    for (int c = 0; c < C; ++c) xd[pt * C + c] = xs[pt * C + c] + d[c];
                }
                __syncthreads();
                cur ^= 1;
            }
        }
        if (cur == 1) {
            for (long long e = tid; e < np * C; e += nt) v.x[e] = v.res[e];
            __syncthreads();
        }
    }
    // up: levels lc - 1 .. 2
    for (int l = lc - 1; l >= 2; --l) {
        const Lev V = level_of(G, l), Cv = level_of(G, l + 1);
        const long long np = (long long)V.lw * V.lw * V.lw;
        const LV<T> v = lvec(l), vc = lvec(l + 1);
        for (long long pt = tid; pt < np; pt += nt) correct_pt<T, C>(G, V, v, vc.x, pt);
        __syncthreads();
        const T *A = Q.A + (P.moff + V.off) * MG_SLOTS * CC;
        const T *D = Q.Dinv + (P.moff + V.off) * MS;
        for (long long pt = tid; pt < np; pt += nt) post_pt<T, C>(G, V, A, D, v, pt);
        __syncthreads();
    }
    // level-2 output to global memory for the level-1 correction
    if (lds && lc >= 2) {
        const Lev V2 = level_of(G, 2);
        const LV<T> g2 = level_vecs<T, C, R>(G, P, w, V2, Q.r, Q.xp, Q.res, Q.x);
        const long long n2 = (long long)V2.lw * V2.lw * V2.lw * C;
        const T *x2 = lvec(2).x;
        for (long long e = tid; e < n2; e += nt) g2.x[e] = x2[e];
    }
}

// Levels 2 .. coarsest when they are small (coarsest level 1, 2 or 3, at most
// MG_FUSED_BS points each; a level-1 coarsest gets only its sweeps): the same
// arithmetic as mg_fused_kernel with the global loads issued up front -- thread t owns level-2 point t and keeps its
// stencil row, l1 inverse and neighbour indices in registers; level-3 stencils,
// inverses and all level >= 2 vectors sit in LDS -- so the kernel waits on
// memory about once instead of once per stage.
template <int C, int R, int BS>
__global__ __launch_bounds__(BS) void mg_fused_small_kernel(const Geo *geos, const Prob *probs,
                                                                     VPtr<float, C, R> Q, int sweeps,
                                                                     const int *prob_active) {
    using T = float;
    constexpr int CC = C * C;
    constexpr int MS = (C == 3) ? 6 : 1;
    extern __shared__ unsigned char mg_smem[];
    const int prob = blockIdx.y, w = blockIdx.x;
    if (prob_active != nullptr && prob_active[prob] == 0) return;
    const Prob &P = probs[prob];
    const Geo &G = geos[P.geo];
    if (G.mg_nlev < 2) return;
    if (P.mg_sweeps > 0) sweeps = P.mg_sweeps;
    const int lc = G.mg_nlev - 1;   // 1, 2 or 3 (checked on the host)
    const int tid = threadIdx.x;
    const Lev V1 = level_of(G, 1);
    const LV<T> g1 = level_vecs<T, C, R>(G, P, w, V1, Q.r, Q.xp, Q.res, Q.x);
    if (lc == 1) {
        // the n/2 grid is the coarsest: sweeps from xp1 with thread t owning point t,
        // its stencil row and inverse in registers, the iterates ping-ponging in LDS
        const int np1 = V1.lw * V1.lw * V1.lw;
        const bool own = tid < np1;
        const int p1 = own ? tid : 0;
        T *const b0 = (T *)mg_smem, *const b1 = b0 + np1 * C;
        T A1[MG_SLOTS * CC], D1[MS], r1[C], x1[C];
        const T *A1g = Q.A + (P.moff + V1.off + p1) * MG_SLOTS * CC;
#pragma unroll
        for (int e = 0; e < MG_SLOTS * CC; ++e) A1[e] = A1g[e];
#pragma unroll
        for (int e = 0; e < MS; ++e) D1[e] = Q.Dinv[(P.moff + V1.off + p1) * MS + e];
        int q1[MG_SLOTS];
        const int *nb1 = row16(G.mg_nbr, V1, p1);
#pragma unroll
        for (int s = 0; s < MG_SLOTS; ++s) q1[s] = nb1[s];
        load_c<T, C>(g1.r + p1 * C, r1);
        load_c<T, C>(g1.xp + p1 * C, x1);
        if (own) store_c<T, C>(b0 + p1 * C, x1);
        __syncthreads();
        int cur = 0;
#pragma unroll 1
        for (int it = 1; it < sweeps; ++it) {
            if (own) {
                const T *xs = cur ? b1 : b0;
                T acc[C];
#pragma unroll
                for (int c = 0; c < C; ++c) acc[c] = r1[c];
#pragma unroll
                for (int s = 0; s < MG_SLOTS; ++s) {
                    T v[C];
                    load_c<T, C>(xs + q1[s] * C, v);
#pragma unroll
                    for (int c = 0; c < C; ++c)
#pragma unroll
                        for (int d = 0; d < C; ++d) acc[c] -= A1[s * CC + c * C + d] * v[d];
                }
                T d[C];
                minv_apply<T, C>(D1, acc, d);
#pragma unroll
                for (int c = 0; c < C; ++c) x1[c] += d[c];
                store_c<T, C>((cur ? b0 : b1) + p1 * C, x1);
            }
            __syncthreads();
            cur ^= 1;
        }
        if (own) store_c<T, C>(g1.x + p1 * C, x1);
        return;
    }
    const Lev V2 = level_of(G, 2);
    const int np2 = V2.lw * V2.lw * V2.lw;
    const LV<T> g2 = level_vecs<T, C, R>(G, P, w, V2, Q.r, Q.xp, Q.res, Q.x);
    // LDS: level 2 xp, res|xc, x (x also the ping-pong partner on a level-2 coarsest);
    // level 3 x, tmp, stencils, inverses (one spare point per vector, kept at zero).
    Lev V3 = V2;
    int np3 = 0;
    if (lc == 3) {
        V3 = level_of(G, 3);
        np3 = V3.lw * V3.lw * V3.lw;
    }
    const int v2 = (np2 + 1) * C, v3 = (np3 + 1) * C;
    T *s2xp = (T *)mg_smem, *s2res = s2xp + v2, *s2x = s2res + v2;
    T *s3x = s2x + v2, *s3t = s3x + v3;
    T *s3A = s3t + v3, *s3D = s3A + np3 * MG_SLOTS * CC;
    if (tid < C) {
        s2xp[np2 * C + tid] = T(0);
        s2res[np2 * C + tid] = T(0);
        s2x[np2 * C + tid] = T(0);
        s3x[np3 * C + tid] = T(0);
        s3t[np3 * C + tid] = T(0);
    }

    // ---- all global loads of the kernel
    const bool own2 = tid < np2;
    const int p2 = own2 ? tid : 0;
    T A2[MG_SLOTS * CC], D2[MS];
    const T *A2g = Q.A + (P.moff + V2.off + p2) * MG_SLOTS * CC;
#pragma unroll
    for (int e = 0; e < MG_SLOTS * CC; ++e) A2[e] = A2g[e];
#pragma unroll
    for (int e = 0; e < MS; ++e) D2[e] = Q.Dinv[(P.moff + V2.off + p2) * MS + e];
    T ch[MG_SLOTS][C];   // level-1 residuals at the children of the owned level-2 point
    T wch[MG_SLOTS];
    const int *chrow = row16(G.mg_child, V2, p2);
#pragma unroll
    for (int m = 0; m < MG_SLOTS; ++m) {
        const int f = chrow[m];
        wch[m] = f < 0 ? T(0) : (m == 0 ? T(1) : T(0.5));
        load_c<T, C>(g1.res + (long long)(f < 0 ? 0 : f) * C, ch[m]);
    }
    if (lc == 3) {
        const T *A3g = Q.A + (P.moff + V3.off) * MG_SLOTS * CC;
        for (int e = tid; e < np3 * MG_SLOTS * CC; e += blockDim.x) s3A[e] = A3g[e];
        const T *D3g = Q.Dinv + (P.moff + V3.off) * MS;
        for (int e = tid; e < np3 * MS; e += blockDim.x) s3D[e] = D3g[e];
    }
    int q2[MG_SLOTS];
    const int *nb2 = row16(G.mg_nbr, V2, p2);
#pragma unroll
    for (int s = 0; s < MG_SLOTS; ++s) q2[s] = nb2[s];

    // ---- restrict 1 -> 2, xp2 = D2^-1 r2
    T r2[C], xp2[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        T a = T(0);
#pragma unroll
        for (int m = 0; m < MG_SLOTS; ++m) a += wch[m] * ch[m][c];
        r2[c] = a;
    }
    minv_apply<T, C>(D2, r2, xp2);
    if (own2) store_c<T, C>(s2xp + p2 * C, xp2);
    __syncthreads();
    // l1 block-Jacobi step on level 2 with the stencil row in registers:
    // out = x_self + D2^-1 (rhs - A2 x)
    auto level2_step = [&](const T *xs, const T rhs[C], const T xself[C], T out[C]) {
        T acc[C];
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = rhs[c];
#pragma unroll
        for (int s = 0; s < MG_SLOTS; ++s) {
            T v[C];
            load_c<T, C>(xs + q2[s] * C, v);
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int d = 0; d < C; ++d) acc[c] -= A2[s * CC + c * C + d] * v[d];
        }
        T d[C];
        minv_apply<T, C>(D2, acc, d);
#pragma unroll
        for (int c = 0; c < C; ++c) out[c] = xself[c] + d[c];
    };
    T x2[C];
    if (lc == 2) {
        // coarsest is level 2: sweeps from xp2, ping-pong between s2x and s2res
        T *const b0 = s2x, *const b1 = s2res;
        if (own2) store_c<T, C>(s2x + p2 * C, xp2);
        __syncthreads();
        int cur = 0;
#pragma unroll 1
        for (int it = 1; it < sweeps; ++it) {
            if (own2) {
                T xs_self[C], o[C];
                const T *xs = cur ? b1 : b0;
                load_c<T, C>(xs + p2 * C, xs_self);
                level2_step(xs, r2, xs_self, o);
                store_c<T, C>((cur ? b0 : b1) + p2 * C, o);
            }
            __syncthreads();
            cur ^= 1;
        }
        load_c<T, C>((cur ? b1 : b0) + p2 * C, x2);
    } else {
        // residual on level 2: res2 = r2 - A2 xp2
        T res2[C];
#pragma unroll
        for (int c = 0; c < C; ++c) res2[c] = r2[c];
#pragma unroll
        for (int s = 0; s < MG_SLOTS; ++s) {
            T v[C];
            load_c<T, C>(s2xp + q2[s] * C, v);
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int d = 0; d < C; ++d) res2[c] -= A2[s * CC + c * C + d] * v[d];
        }
        if (own2) store_c<T, C>(s2res + p2 * C, res2);
        __syncthreads();
        // restrict 2 -> 3 and the coarsest sweeps (threads < np3)
        const bool own3 = tid < np3;
        const int p3 = own3 ? tid : 0;
        int q3[MG_SLOTS];
        const int *nb3 = row16(G.mg_nbr, V3, p3);
#pragma unroll
        for (int s = 0; s < MG_SLOTS; ++s) q3[s] = nb3[s];
        T r3[C], D3[MS];
#pragma unroll
        for (int c = 0; c < C; ++c) r3[c] = T(0);
        const int *ch3 = row16(G.mg_child, V3, p3);
#pragma unroll
        for (int m = 0; m < MG_SLOTS; ++m) {
            const int f = ch3[m];
            const T wgt = f < 0 ? T(0) : (m == 0 ? T(1) : T(0.5));
            const int fs = f < 0 ? 0 : f;
#pragma unroll
            for (int c = 0; c < C; ++c) r3[c] += wgt * s2res[fs * C + c];
        }
#pragma unroll
        for (int e = 0; e < MS; ++e) D3[e] = s3D[p3 * MS + e];
        T xp3[C];
        minv_apply<T, C>(D3, r3, xp3);
        if (own3) store_c<T, C>(s3x + p3 * C, xp3);
        __syncthreads();
        T *const b0 = s3x, *const b1 = s3t;
        int cur = 0;
        const T *A3 = s3A + p3 * MG_SLOTS * CC;
#pragma unroll 1
        for (int it = 1; it < sweeps; ++it) {
            if (own3) {
                const T *xs = cur ? b1 : b0;
                T acc[C];
#pragma unroll
                for (int c = 0; c < C; ++c) acc[c] = r3[c];
#pragma unroll
                for (int s = 0; s < MG_SLOTS; ++s) {
                    T v[C];
                    load_c<T, C>(xs + q3[s] * C, v);
#pragma unroll
                    for (int c = 0; c < C; ++c)
#pragma unroll
                        for (int d = 0; d < C; ++d) acc[c] -= A3[s * CC + c * C + d] * v[d];
                }
                T d[C], xo[C];
                minv_apply<T, C>(D3, acc, d);
                load_c<T, C>(xs + p3 * C, xo);
#pragma unroll
                for (int c = 0; c < C; ++c) (cur ? b0 : b1)[p3 * C + c] = xo[c] + d[c];
            }
            __syncthreads();
            cur ^= 1;
        }
        const T *e3 = cur ? b1 : b0;
        // correct and post-smooth level 2
        T xc2[C], pe[C];
        prolong<T, C>(G, V2, e3, p2, pe);
#pragma unroll
        for (int c = 0; c < C; ++c) xc2[c] = xp2[c] + pe[c];
        if (own2) store_c<T, C>(s2res + p2 * C, xc2);
        __syncthreads();
        level2_step(s2res, r2, xc2, x2);
    }
    if (own2) store_c<T, C>(g2.x + p2 * C, x2);
}

// Fine vector of constraint columns for the Gram setup: load case w carries the
// column (i, a) = (s / nrow, s % nrow), s = first + w: component i equals row a.
template <typename T, int C, int R>
__global__ __launch_bounds__(64 * R) void mg_cols_kernel(const Geo *geos, const Prob *probs, int first, T *v) {
    const int prob = blockIdx.y;
    const Prob &P = probs[prob];
    const Geo &G = geos[P.geo];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nr = G.nrow, rf = row_first(G.nrow);
    const int s = first + w;
    const int ci = nr > 0 ? s / nr : C, a = nr > 0 ? s % nr : 0;
    const long long nblk = (G.npts + 63) / 64;
    for (long long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const long long pt = blk * 64 + lane;
        if (pt >= G.npts) continue;
        T *dst = v + P.voff + ((long long)w * G.npts + pt) * C;
#pragma unroll
        for (int c = 0; c < C; ++c) dst[c] = (c == ci) ? (T)G.rows[4 * pt + rf + a] : T(0);
    }
}

// W[level-1 point][i * 4 + a] = level-1 output of the column batch.
template <typename T, int C, int R>
__global__ void mg_store_w_kernel(const Geo *geos, const Prob *probs, int first, const T *lx, T *W) {
    const int prob = blockIdx.y;
    const Prob &P = probs[prob];
    const Geo &G = geos[P.geo];
    if (G.mg_nlev < 2 || G.nrow == 0) return;
    const int nr = G.nrow;
    const Lev V = level_of(G, 1);
    const long long np1 = (long long)V.lw * V.lw * V.lw;
    for (long long u = blockIdx.x * (long long)blockDim.x + threadIdx.x; u < np1 * R;
         u += (long long)gridDim.x * blockDim.x) {
        const int w = (int)(u / np1);
        const long long v = u - (long long)w * np1;
        const int s = first + w;
        if (s >= C * nr) continue;
        const int i = s / nr, a = s % nr;
        const T *src = lx + (P.moff * R + (long long)w * G.mg_pts + V.off + v) * C;
        T *dst = W + ((P.moff + V.off + v) * (4 * C) + i * 4 + a) * C;
#pragma unroll
        for (int c = 0; c < C; ++c) dst[c] = src[c];
    }
}

// E[(i,a),(j,b)] = sum over level-1 points of rows1_a W[.][j*4+b][i]; partials per workgroup.
template <int C, typename T>
__global__ void mg_gram_partial_kernel(const Geo *geos, const Prob *probs, const T *W, const double *rows1,
                                       double *partial) {
    const int prob = blockIdx.y;
    const Prob &P = probs[prob];
    const Geo &G = geos[P.geo];
    double *out = partial + ((long long)prob * gridDim.x + blockIdx.x) * 144;
    const int nr = G.nrow, S = C * nr, rf = row_first(G.nrow);
    const int u = threadIdx.x;
    if (G.mg_nlev < 2 || nr == 0) {
        if (u < 144) out[u] = 0.0;
        return;
    }
    double acc = 0.0;
    if (u < S * S) {
        const int I = u / S, J = u % S;
        const int i = I / nr, a = I % nr, j = J / nr, b = J % nr;
        const Lev V = level_of(G, 1);
        const long long np1 = (long long)V.lw * V.lw * V.lw;
        for (long long v = blockIdx.x; v < np1; v += gridDim.x)
            acc += rows1[(P.moff + V.off + v) * 4 + rf + a] *
                   (double)W[((P.moff + V.off + v) * (4 * C) + j * 4 + b) * C + i];
    }
    if (u < 144) out[u] = acc;
}

// G_B = G_M + E, inverted (one workgroup per problem).
template <int C>
__global__ __launch_bounds__(256) void mg_gram_finish_kernel(const Geo *geos, const Prob *probs, int nwg,
                                                             const double *partial, const double *gmat,
                                                             double *ginv, int *bad) {
    constexpr int SMAX = C * 4;
    __shared__ double A[12][24];
    __shared__ int ok_s, piv_s[2];
    const int prob = blockIdx.x;
    const Geo &G = geos[probs[prob].geo];
    const int nr = G.nrow, S = C * nr;
    if (nr == 0) return;
    for (int t = threadIdx.x; t < S * S; t += blockDim.x) {
        const int I = t / S, J = t % S;
        double e = 0.0;
        if (G.mg_nlev >= 2)
            for (int b = 0; b < nwg; ++b) e += partial[((long long)prob * nwg + b) * 144 + t];
        A[I][J] = gmat[(long long)prob * SMAX * SMAX + t] + e;
        A[I][S + J] = (I == J) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int ok = gauss_jordan_wg(A, S, piv_s);
    if (threadIdx.x == 0) {
        ok_s = ok;
        if (!ok) atomicAdd(bad, 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < S * S; t += blockDim.x)
        ginv[(long long)prob * SMAX * SMAX + t] = ok_s ? A[t / S][S + t % S] : 0.0;
}

// Load cases per lane in the level-1 kernels: for launches over many problems
// three where they divide the cases (fewer waves reload each stencil block;
// mechanics 6 cases: 475 -> 477 homogenisations/s on the 512-record mixed
// batch against two), for a few problems two (more waves per problem: the
// three-problem 24^3 batch 192 -> 197/s against three).
template <int R> constexpr int MG_KG_MANY = R % 3 == 0 ? 3 : (R % 2 == 0 ? 2 : 1);
template <int R> constexpr int MG_KG_FEW = R % 2 == 0 ? 2 : (R % 3 == 0 ? 3 : 1);
constexpr int MG_MANY_PROBLEMS = 16;

// Calls f with std::integral_constant<int, KG> for the launch's problem count.
template <int R, typename F>
static void with_mg_kg(int nprob, F &&f) {
    if (nprob >= MG_MANY_PROBLEMS)
        f(std::integral_constant<int, MG_KG_MANY<R>>{});
    else
        f(std::integral_constant<int, MG_KG_FEW<R>>{});
}

#define CHOM_MG_NR_DISPATCH(NRV, CALL)                 \
    switch (NRV) {                                     \
        case 0: { constexpr int NR = 0; CALL; } break; \
        case 1: { constexpr int NR = 1; CALL; } break; \
        default: { constexpr int NR = 4; CALL; } break; \
    }

}  // namespace

// ------------------------------------------------------------------ launchers
template <typename T, int C>
hipError_t launch_mg_stencils(const Launch &L, T *A, T *Dinv, hipStream_t s) {
    constexpr int CC = C * C;
    constexpr int MS = (C == 3) ? 6 : 1;
    const auto &M = L.mg;
    mg_assemble0_kernel<C><<<dim3(grid_cap(M.max_pts[0] * MG_SLOTS, MG_BS, 4096), L.nprob), MG_BS, 0, s>>>(
        L.geos, L.probs, M.A64);
    for (int l = 0; l + 1 < M.nlev; ++l)
        mg_rap_kernel<C><<<dim3(grid_cap(M.max_pts[l + 1] * MG_SLOTS, MG_BS, 4096), L.nprob), MG_BS, 0, s>>>(
            L.geos, L.probs, l, M.A64);
    mg_dinv_kernel<C><<<grid_cap(M.total_pts, MG_BS, 8192), MG_BS, 0, s>>>(M.total_pts, M.A64, M.D64);
    mg_rows1_kernel<<<dim3(grid_cap(M.max_pts[1], MG_BS, 1024), L.nprob), MG_BS, 0, s>>>(L.geos, L.probs, M.rows1);
    if constexpr (std::is_same<T, float>::value) {
        mg_to_float_kernel<<<grid_cap(M.total_pts * MG_SLOTS * CC, MG_BS, 8192), MG_BS, 0, s>>>(
            M.total_pts * MG_SLOTS * CC, M.A64, A);
        mg_to_float_kernel<<<grid_cap(M.total_pts * MS, MG_BS, 8192), MG_BS, 0, s>>>(M.total_pts * MS, M.D64, Dinv);
    }
    return hipGetLastError();
}

template <typename T, int C, int R>
hipError_t launch_mg_vcycle(const Launch &L, const T *r, double *accbuf, const int *prob_active, hipStream_t s) {
    const auto &M = L.mg;
    VPtr<T, C, R> Q;
    Q.fine_r = r;
    Q.A = (const T *)M.A;
    Q.Dinv = (const T *)M.Dinv;
    Q.r = (T *)M.r;
    Q.xp = (T *)M.xp;
    Q.res = (T *)M.res;
    Q.x = (T *)M.x;
    Q.rows1 = M.rows1;
    const dim3 g1(M.nwg[1], L.nprob);
    with_mg_kg<R>(L.nprob, [&](auto kg) {
        constexpr int KG = decltype(kg)::value;
        mg_restrict01_kernel<T, C, R, KG><<<g1, 64 * (R / KG), 0, s>>>(L.geos, L.probs, Q, prob_active);
        mg_resid1_kernel<T, C, R, KG><<<g1, 64 * (R / KG), 0, s>>>(L.geos, L.probs, Q, prob_active);
    });
    if constexpr (std::is_same<T, float>::value) {
        if (M.small_elems > 0) {
            // thread t owns point t of the level-1 (coarsest) or level-2 grid: 256 threads
            // when every owned level has at most 256 points, else 512
            if (M.small_bs == 256)
                mg_fused_small_kernel<C, R, 256><<<dim3(R, L.nprob), 256, (size_t)M.small_elems * sizeof(float), s>>>(
                    L.geos, L.probs, Q, M.sweeps, prob_active);
            else
                mg_fused_small_kernel<C, R, MG_FUSED_BS><<<dim3(R, L.nprob), MG_FUSED_BS,
                                                           (size_t)M.small_elems * sizeof(float), s>>>(
                    L.geos, L.probs, Q, M.sweeps, prob_active);
        } else {
            mg_fused_kernel<T, C, R><<<dim3(R, L.nprob), MG_FUSED_BS, (size_t)M.lds_elems * sizeof(T), s>>>(
                L.geos, L.probs, Q, M.sweeps, M.lds_vec, M.lds_sten, prob_active);
        }
    } else {
        mg_fused_kernel<T, C, R><<<dim3(R, L.nprob), MG_FUSED_BS, (size_t)M.lds_elems * sizeof(T), s>>>(
            L.geos, L.probs, Q, M.sweeps, M.lds_vec, M.lds_sten, prob_active);
    }
    with_mg_kg<R>(L.nprob, [&](auto kg) {
        constexpr int KG = decltype(kg)::value;
        mg_correct1_kernel<T, C, R, KG><<<g1, 64 * (R / KG), 0, s>>>(L.geos, L.probs, Q, prob_active);
        CHOM_MG_NR_DISPATCH(L.nr, (mg_post1_kernel<T, C, R, NR, KG><<<g1, 64 * (R / KG), 0, s>>>(
                                      L.geos, L.probs, Q, accbuf, prob_active)));
    });
    return hipGetLastError();
}

template <typename T, int C, int R>
hipError_t launch_mg_fcorr(const Launch &L, const double *ycoef, const int *prob_active, hipStream_t s) {
    const auto &M = L.mg;
    VPtr<T, C, R> Q;
    Q.fine_r = nullptr;
    Q.A = (const T *)M.A;
    Q.Dinv = (const T *)M.Dinv;
    Q.r = (T *)M.r;
    Q.xp = (T *)M.xp;
    Q.res = (T *)M.res;
    Q.x = (T *)M.x;
    Q.rows1 = M.rows1;
    with_mg_kg<R>(L.nprob, [&](auto kg) {
        constexpr int KG = decltype(kg)::value;
        CHOM_MG_NR_DISPATCH(L.nr, (mg_fcorr_kernel<T, C, R, NR, KG><<<dim3(M.nwg[1], L.nprob), 64 * (R / KG), 0, s>>>(
                                      L.geos, L.probs, Q, (const T *)M.W, ycoef, prob_active)));
    });
    return hipGetLastError();
}

template <typename T, int C, int R>
hipError_t launch_mg_gram(const Launch &L, T *tmp, const double *gmat, double *partial, int nwg, double *ginv,
                          int *bad, hipStream_t s) {
    if (L.nr == 0) return hipSuccess;
    const auto &M = L.mg;
    const int S = C * 4;
    for (int first = 0; first < S; first += R) {
        mg_cols_kernel<T, C, R><<<dim3(L.nwg, L.nprob), 64 * R, 0, s>>>(L.geos, L.probs, first, tmp);
        hipError_t e = launch_mg_vcycle<T, C, R>(L, tmp, nullptr, nullptr, s);
        if (e != hipSuccess) return e;
        mg_store_w_kernel<T, C, R><<<dim3(grid_cap(M.max_pts[1] * R, MG_BS, 1024), L.nprob), MG_BS, 0, s>>>(
            L.geos, L.probs, first, (const T *)M.x, (T *)M.W);
    }
    mg_gram_partial_kernel<C, T><<<dim3(nwg, L.nprob), 192, 0, s>>>(L.geos, L.probs, (const T *)M.W, M.rows1, partial);
    mg_gram_finish_kernel<C><<<L.nprob, 256, 0, s>>>(L.geos, L.probs, nwg, partial, gmat, ginv, bad);
    return hipGetLastError();
}

#define CHOM_MG_INST(T, C, R)                                                                                    \
    template hipError_t launch_mg_vcycle<T, C, R>(const Launch &, const T *, double *, const int *, hipStream_t); \
    template hipError_t launch_mg_fcorr<T, C, R>(const Launch &, const double *, const int *, hipStream_t);      \
    template hipError_t launch_mg_gram<T, C, R>(const Launch &, T *, const double *, double *, int, double *,    \
                                                int *, hipStream_t);
CHOM_MG_INST(float, 3, 6)
CHOM_MG_INST(float, 1, 3)
CHOM_MG_INST(double, 3, 6)
CHOM_MG_INST(double, 1, 3)
template hipError_t launch_mg_stencils<float, 3>(const Launch &, float *, float *, hipStream_t);
template hipError_t launch_mg_stencils<float, 1>(const Launch &, float *, float *, hipStream_t);
template hipError_t launch_mg_stencils<double, 3>(const Launch &, double *, double *, hipStream_t);
template hipError_t launch_mg_stencils<double, 1>(const Launch &, double *, double *, hipStream_t);

}  // namespace chom
