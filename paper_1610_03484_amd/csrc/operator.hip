// Matrix-free stiffness / conductivity operator Y = K X for the order-2
// hierarchic space on the Kuhn lattice (K is the standard FE matrix of Sec. 2,
// Eq. eq_RVE_disc_Eqs, and its scalar analogue, Eq. eq_RVE_disc_Eqs_field).
//
// One workgroup owns a tile of TX x TY x TZ cells (6 tets each, one thread per
// tet) and one group of RG load cases.  It stages the (2T+1)^3 DOF box of its
// tile from HBM into LDS (all loads in flight before the first LDS store),
// applies every tet of the tile (element data: fibre axis + phase, 16/32 bytes;
// the stiffness is evaluated on the fly from five invariants), accumulates the
// element results in an FP64 LDS box with LDS atomics (FP64 LDS atomic adds are
// markedly faster than FP32 ones on gfx950), and stores the whole box,
// contiguous and load-case major, to its slot of the tile-box output: no
// global atomics, no zeroing pass; consumers sum the copies of points on shared
// tile faces.  The element
// energies x_e . K_e x_e (p.Kp for CG) are formed per tet in the vector
// precision and summed in FP64.
//
// Problems of different RVEs (sizes, BCs) share a launch: grid.x covers the
// largest problem's tiles x groups; workgroups past a problem's tiles only
// write zero partials.
#include "common.h"
#include "internal.h"

#include <type_traits>

namespace chom {

int operator_tiles(const Geo &G) { return G.tiles_x * G.tiles_y * G.tiles_z; }

// MODE: OP_APPLY  y = K x (and the element energies x.Kx);
//       OP_RHS    no input vector; every tet applies its constant stress (flux)
//                 of the unit macro strain (gradient) of the load case,
//                 y = int grad(phi) . C eps_k, and its energy |e| eps_k . C eps_k
//                 goes to the accumulators (load vectors of the fluctuation
//                 problems, Sec. 2, Eqs. Eq_C_stress and eq_homo_flux);
//       OP_DIAG   (FP64, group 0 only; RG C = 6 for elasticity, 1 for the scalar
//                 fields) the point blocks of diag(K): per node the element's
//                 block int grad(phi) C grad(phi), packed xx yy zz | xy yz xz in
//                 the group's RG C slots.
enum { OP_APPLY = 0, OP_RHS = 1, OP_DIAG = 2 };
template <typename T, int C, int R, int RG, int MODE = OP_APPLY>
__global__ __launch_bounds__(TILE_TETS) void op_p2_kernel(const Geo *geos, const Prob *probs, int max_tiles,
                                                          const T *__restrict__ x, T *__restrict__ y,
                                                          double *acc_pq, const int *prob_active) {
    constexpr bool RHS = MODE == OP_RHS, DIAG = MODE == OP_DIAG, STAGE = MODE == OP_APPLY;
    static_assert(!DIAG || (std::is_same<T, double>::value && RG * C == (C == 3 ? 6 : 1)), "diag mode layout");
    constexpr int NG = R / RG;
    constexpr int RCg = RG * C;
    // LDS layout of the box: point (bx, by, bz) at bx + BXP (by + BY bz), PS
    // values per point.  Neighbouring tets of a wave sit two lattice points apart,
    // so an even point stride maps them onto few banks; an odd PS and a row pitch
    // of 10 (12 for narrow FP32 boxes) keep the per-node LDS reads and FP64
    // atomics of a wave at about two passes per 32 lanes.
    constexpr int PS = RCg | 1;
    constexpr int BXP = (sizeof(T) == 4 && RCg <= 3) ? 12 : 10;
    constexpr int LPTS = BXP * BY * BZ;
    constexpr int NBOX = BOXPTS * RCg;
    constexpr int NCELL = TX * TY * TZ;
    constexpr int NW = TILE_TETS / 64;
    using V4 = typename std::conditional<std::is_same<T, double>::value, double4, float4>::type;
    __shared__ T xs[LPTS * PS];
    __shared__ double ys[LPTS * PS];
    __shared__ T sg[6][10];
    __shared__ double red[RG][NW];
    const int prob = blockIdx.y;
    const int tile = DIAG ? (int)blockIdx.x : (int)blockIdx.x / NG;
    const int grp = DIAG ? 0 : (int)blockIdx.x - ((int)blockIdx.x / NG) * NG;
    const int tt = threadIdx.x;
    const Prob &P = probs[prob];
    const Geo &G = geos[P.geo];
    if (tile >= G.ntiles || (prob_active != nullptr && prob_active[prob] == 0)) return;
    const int n = G.n, m2 = 2 * n;
    const int tx = tile % G.tiles_x, ty = (tile / G.tiles_x) % G.tiles_y, tz = tile / (G.tiles_x * G.tiles_y);
    const int cx0 = tx * TX, cy0 = ty * TY, cz0 = tz * TZ;
    const int X0 = 2 * cx0, Y0 = 2 * cy0, Z0 = 2 * cz0;
    const int hx = min(X0 + 2 * TX, m2), hy = min(Y0 + 2 * TY, m2), hz = min(Z0 + 2 * TZ, m2);
    const T *xp = STAGE ? x + P.voff : nullptr;   // vectors are [load case][point][component]

    // ---- stage the DOF box (this group's values), element data, geometry.
    // The box is RG x BY x BZ rows of BX points x C values, each row contiguous
    // in the lattice: thread tt takes column tt % ROWLEN of rows tt / ROWLEN +
    // RPP k, so its x coordinate, periodic wrap and LDS column are fixed and only
    // a row offset changes per pass.  Every load is issued unconditionally
    // (out-of-box elements read element 0 and are replaced by zero), all NPASS
    // loads in flight together.
    constexpr int ROWLEN = BX * C;
    constexpr int NROW = RG * BY * BZ;
    constexpr int RPP = TILE_TETS / ROWLEN;   // rows per pass
    constexpr int NPASS = (NROW + RPP - 1) / RPP;
    const int col = tt % ROWLEN, r0 = tt / ROWLEN;
    const bool colok = r0 < RPP;
    const int bxc = col / C, cc = col - (col / C) * C;
    const int colL = bxc * PS + cc;   // LDS offset of the column within a box row
    T tmp[NPASS];
    if constexpr (STAGE) {
        const int Lw = G.Lw, Lm = (G.bc == 1) ? G.L : -1;   // periodic: index L wraps to 0
        const long long np = G.npts;
        const T *xg = xp + (long long)grp * RG * np * C;
        const int Xc = X0 + bxc;
        const bool inx = colok && Xc <= hx;
        const int Xw = Xc == Lm ? 0 : Xc;
#pragma unroll
        for (int k = 0; k < NPASS; ++k) {
            const int row = r0 + RPP * k;
            const int rr = row / (BY * BZ), rem = row - rr * (BY * BZ);
            const int bz = rem / BY, by = rem - (rem / BY) * BY;
            int Y = Y0 + by, Z = Z0 + bz;
            const bool in = inx && row < NROW && Y <= hy && Z <= hz;
            Y = Y == Lm ? 0 : Y;
            Z = Z == Lm ? 0 : Z;
            const long long idx = in ? ((long long)rr * np + Xw + (long long)Lw * (Y + Lw * Z)) * C + cc : 0;
            const T v = xg[idx];
            tmp[k] = in ? v : T(0);
        }
    }
    const int type = tt / NCELL, lc = tt - (tt / NCELL) * NCELL;
    const int lcx = lc % TX, lcy = (lc / TX) % TY, lcz = lc / (TX * TY);
    const int ci = cx0 + lcx, cj = cy0 + lcy, ck = cz0 + lcz;
    const bool live = (ci < n && cj < n && ck < n);
    const long long tet = ((long long)ci + (long long)n * (cj + (long long)n * ck)) * 6 + type;
    V4 ev;
    if (live) {
        if constexpr (std::is_same<T, double>::value) ev = G.elem64[tet]; else ev = G.elem32[tet];
    }
    if constexpr (STAGE) {
#pragma unroll
        for (int k = 0; k < NPASS; ++k) {
            const int row = r0 + RPP * k;
            if (colok && row < NROW) {
                const int rr = row / (BY * BZ), rem = row - rr * (BY * BZ);
                xs[BXP * rem * PS + rr * C + colL] = tmp[k];   // rem = by + BY bz
            }
        }
    }
    for (int i = tt; i < LPTS * PS; i += TILE_TETS) ys[i] = 0.0;
    if (tt < 60 && G.uniform) {
        if constexpr (std::is_same<T, double>::value) sg[tt / 10][tt % 10] = G.tg64[tt / 10][tt % 10];
        else sg[tt / 10][tt % 10] = G.tg32[tt / 10][tt % 10];
    }
    __syncthreads();

    // ---- element work: one tet per thread, the group's load cases in turn
    double pq[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) pq[r] = 0.0;
    if (live) {
        T g[4][3], vol, a[3];
        if (G.uniform) {
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) g[i + 1][j] = sg[type][3 * i + j];
            vol = sg[type][9];
#pragma unroll
            for (int j = 0; j < 3; ++j) g[0][j] = -(g[1][j] + g[2][j] + g[3][j]);
        } else {
            GeoSel<T>::get(G, tet, type, g, vol);
        }
        a[0] = ev.x; a[1] = ev.y; a[2] = ev.z;
        const T *mt = prob_mat<T>(P, (int)ev.w);
        T mloc[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) mloc[k] = mt[k];
        int off[10][3];
        p2_dof_offsets(type, off);
        int lp[10];
#pragma unroll
        for (int k = 0; k < 10; ++k)
            lp[k] = ((2 * lcx + off[k][0]) + BXP * ((2 * lcy + off[k][1]) + BY * (2 * lcz + off[k][2]))) * PS;
        if constexpr (DIAG) {
            // vertex a: |e| Q(g_a); edge (a, b): (4/5)|e| [Q(g_a + g_b) + Q(g_a) + Q(g_b)],
            // Q(w) = sum_kl C_.k.l w_k w_l (the integrals of the hierarchic basis products)
#pragma unroll 1
            for (int k = 0; k < 10; ++k) {
                double ws[3][3], cs;
                int nw;
                if (k < 4) {
                    nw = 1;
                    for (int d = 0; d < 3; ++d) ws[0][d] = g[k][d];
                    cs = vol;
                } else {
                    int a2, b2;
                    edge_verts(k - 4, a2, b2);
                    nw = 3;
                    for (int d = 0; d < 3; ++d) {
                        ws[0][d] = g[a2][d] + g[b2][d];
                        ws[1][d] = g[a2][d];
                        ws[2][d] = g[b2][d];
                    }
                    cs = 0.8 * vol;
                }
                if constexpr (C == 3) {
                    double acc[6] = {0, 0, 0, 0, 0, 0};
                    for (int q = 0; q < nw; ++q) {
                        double Q[3][3];
                        acoustic(ws[q], a, mloc, Q);
                        acc[0] += cs * Q[0][0];
                        acc[1] += cs * Q[1][1];
                        acc[2] += cs * Q[2][2];
                        acc[3] += cs * Q[0][1];
                        acc[4] += cs * Q[1][2];
                        acc[5] += cs * Q[0][2];
                    }
#pragma unroll
                    for (int v = 0; v < 6; ++v) atomicAdd(&ys[lp[k] + v], acc[v]);
                } else {
                    double acc = 0.0;
                    for (int q = 0; q < nw; ++q) {
                        double fl[3];
                        flux_ti<double>(ws[q], a, mloc, fl);
                        acc += cs * (fl[0] * ws[q][0] + fl[1] * ws[q][1] + fl[2] * ws[q][2]);
                    }
                    atomicAdd(&ys[lp[k]], acc);
                }
            }
        } else {
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            T yv[10][C];
            double en = 0.0;
            if constexpr (RHS) {
                // constant stress of the unit load case: y_a = |e| sigma g_a, y_ab = |e| sigma (g_a + g_b)
                const int kc = grp * RG + r;
                T sv[3][3];
                if constexpr (C == 3) {
                    T eps[6] = {0, 0, 0, 0, 0, 0};
                    eps[kc] = kc < 3 ? T(1) : T(0.5);   // engineering shear 1
                    T sgm[6];
                    stress_ti<T>(eps, a, mloc, sgm);
                    sv[0][0] = sgm[0]; sv[0][1] = sgm[3]; sv[0][2] = sgm[5];
                    sv[1][0] = sgm[3]; sv[1][1] = sgm[1]; sv[1][2] = sgm[4];
                    sv[2][0] = sgm[5]; sv[2][1] = sgm[4]; sv[2][2] = sgm[2];
                    en = (double)vol * (double)sgm[kc];
                } else {
                    T gk[3] = {0, 0, 0};
                    gk[kc] = T(1);
                    T fl[3];
                    flux_ti<T>(gk, a, mloc, fl);
                    sv[0][0] = fl[0]; sv[0][1] = fl[1]; sv[0][2] = fl[2];
                    en = (double)vol * (double)fl[kc];
                }
#pragma unroll
                for (int k = 0; k < 10; ++k) {
                    T w3[3];
                    if (k < 4) {
#pragma unroll
                        for (int d = 0; d < 3; ++d) w3[d] = vol * g[k][d];
                    } else {
                        int ea, eb;
                        edge_verts(k - 4, ea, eb);
#pragma unroll
                        for (int d = 0; d < 3; ++d) w3[d] = vol * (g[ea][d] + g[eb][d]);
                    }
#pragma unroll
                    for (int c = 0; c < C; ++c) yv[k][c] = sv[c][0] * w3[0] + sv[c][1] * w3[1] + sv[c][2] * w3[2];
                }
            } else {
                T u[10][C];
#pragma unroll
                for (int k = 0; k < 10; ++k)
#pragma unroll
                    for (int c = 0; c < C; ++c) u[k][c] = xs[lp[k] + r * C + c];
                p2_apply<T, C>(g, vol, a, mloc, u, yv);
                // element energy in the vector precision (one FP64 conversion per tet)
                T et = T(0);
#pragma unroll
                for (int k = 0; k < 10; ++k)
#pragma unroll
                    for (int c = 0; c < C; ++c) et += u[k][c] * yv[k][c];
                en = (double)et;
            }
#pragma unroll
            for (int k = 0; k < 10; ++k)
#pragma unroll
                for (int c = 0; c < C; ++c) atomicAdd(&ys[lp[k] + r * C + c], (double)yv[k][c]);
            pq[r] = en;
        }
        }
    }
    __syncthreads();

    // ---- write this group's tile box (load-case major, rows contiguous)
    T *qt = y + P.qoff + ((long long)tile * NG + grp) * NBOX;
#pragma unroll
    for (int k = 0; k < NPASS; ++k) {
        const int row = r0 + RPP * k;
        if (colok && row < NROW) {
            const int rr = row / (BY * BZ), rem = row - rr * (BY * BZ);   // rem = by + BY bz
            qt[(rr * BOXPTS + BX * rem) * C + col] = (T)ys[BXP * rem * PS + rr * C + colL];
        }
    }

    // ---- element energies p.Kp into the striped accumulators [prob][load case][ACC_STRIPES]
    if constexpr (DIAG) return;
    const int lane = tt & 63, wv = tt >> 6;
#pragma unroll
    for (int r = 0; r < RG; ++r) {
        const double s = wave_sum(pq[r]);
        if (lane == 0) red[r][wv] = s;
    }
    __syncthreads();
    if (tt < RG) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += red[tt][w];
        unsafeAtomicAdd(&acc_pq[((long long)prob * R + grp * RG + tt) * ACC_STRIPES + (tile & (ACC_STRIPES - 1))], s);
    }
}

template <typename T, int C, int R, int RG>
static hipError_t launch_rg(const Geo *geos, const Prob *probs, int nprob, int max_tiles, const T *x, T *y,
                            double *acc_pq, const int *prob_active, hipStream_t s) {
    dim3 grid(max_tiles * (R / RG), nprob);
    op_p2_kernel<T, C, R, RG><<<grid, TILE_TETS, 0, s>>>(geos, probs, max_tiles, x, y, acc_pq, prob_active);
    return hipGetLastError();
}

// Tile boxes of K x_lin for the unit load cases (FP64, grouping rg) and the
// linear-field energies in acc_pq.
template <int C, int R>
hipError_t launch_rhs_operator(const Launch &L, int rg, double *y, double *acc_pq, hipStream_t s) {
    const int G = L.max_tiles;
    if constexpr (C == 3) {
        switch (rg) {
            case 1: op_p2_kernel<double, C, R, 1, OP_RHS><<<dim3(G * R, L.nprob), TILE_TETS, 0, s>>>(L.geos, L.probs, G, nullptr, y, acc_pq, nullptr); break;
            case 3: op_p2_kernel<double, C, R, 3, OP_RHS><<<dim3(G * (R / 3), L.nprob), TILE_TETS, 0, s>>>(L.geos, L.probs, G, nullptr, y, acc_pq, nullptr); break;
            default: op_p2_kernel<double, C, R, 2, OP_RHS><<<dim3(G * (R / 2), L.nprob), TILE_TETS, 0, s>>>(L.geos, L.probs, G, nullptr, y, acc_pq, nullptr); break;
        }
    } else {
        switch (rg) {
            case 1: op_p2_kernel<double, C, R, 1, OP_RHS><<<dim3(G * R, L.nprob), TILE_TETS, 0, s>>>(L.geos, L.probs, G, nullptr, y, acc_pq, nullptr); break;
            default: op_p2_kernel<double, C, R, 3, OP_RHS><<<dim3(G * (R / 3), L.nprob), TILE_TETS, 0, s>>>(L.geos, L.probs, G, nullptr, y, acc_pq, nullptr); break;
        }
    }
    return hipGetLastError();
}
template hipError_t launch_rhs_operator<3, 6>(const Launch &, int, double *, double *, hipStream_t);
template hipError_t launch_rhs_operator<1, 3>(const Launch &, int, double *, double *, hipStream_t);

// Tile boxes (group 0, FP64) of the point blocks of diag(K), order 2.
template <int C, int R>
hipError_t launch_diag_operator(const Launch &L, double *y, hipStream_t s) {
    constexpr int RG = (C == 3) ? 2 : 1;
    op_p2_kernel<double, C, R, RG, OP_DIAG><<<dim3(L.max_tiles, L.nprob), TILE_TETS, 0, s>>>(
        L.geos, L.probs, L.max_tiles, nullptr, y, nullptr, nullptr);
    return hipGetLastError();
}
template hipError_t launch_diag_operator<3, 6>(const Launch &, double *, hipStream_t);
template hipError_t launch_diag_operator<1, 3>(const Launch &, double *, hipStream_t);

template <typename T, int C, int R>
hipError_t launch_operator(const Launch &L, int nprob, int rg, const T *x, T *y, double *acc_pq,
                           const int *prob_active, hipStream_t s) {
    if (L.order != 2) return launch_operator_hp<T, C, R>(L, nprob, rg, x, y, acc_pq, prob_active, s);
    const Geo *geos = L.geos;
    const Prob *probs = L.probs;
    const int max_tiles = L.max_tiles;
    if constexpr (C == 3) {
        switch (rg) {
            case 1: return launch_rg<T, C, R, 1>(geos, probs, nprob, max_tiles, x, y, acc_pq, prob_active, s);
            case 3: return launch_rg<T, C, R, 3>(geos, probs, nprob, max_tiles, x, y, acc_pq, prob_active, s);
            default: return launch_rg<T, C, R, 2>(geos, probs, nprob, max_tiles, x, y, acc_pq, prob_active, s);
        }
    } else {
        switch (rg) {
            case 1: return launch_rg<T, C, R, 1>(geos, probs, nprob, max_tiles, x, y, acc_pq, prob_active, s);
            default: return launch_rg<T, C, R, 3>(geos, probs, nprob, max_tiles, x, y, acc_pq, prob_active, s);
        }
    }
}

template hipError_t launch_operator<double, 3, 6>(const Launch &, int, int, const double *, double *, double *, const int *, hipStream_t);
template hipError_t launch_operator<float, 3, 6>(const Launch &, int, int, const float *, float *, double *, const int *, hipStream_t);
template hipError_t launch_operator<double, 1, 3>(const Launch &, int, int, const double *, double *, double *, const int *, hipStream_t);
template hipError_t launch_operator<float, 1, 3>(const Launch &, int, int, const float *, float *, double *, const int *, hipStream_t);

}  // namespace chom
