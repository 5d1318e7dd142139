// Orders p = 3, 4: setup kernels and the element-batched operator.
//
// K_e of Sec. 2 (Eq. eq_RVE_disc_Eqs; Eq. eq_RVE_disc_Eqs_field for the scalar
// fields) for the order-p hierarchic space, applied as
//   y_e = sum_k D_k^T [ sum_l Q_e^{kl} (D_l x_e) ],
//   Q_e^{kl}_{cd} = |e| sum_mn (grad lam_k)_m C_{cmdn} (grad lam_l)_n   (k, l = 1..3),
// where D_k are the order's derivative tables in a mass-orthonormal basis of
// P_{p-1} (shared by every tet).  Q_e is precomputed per problem and tet (the
// element factors, 45 or 6 numbers).  A workgroup takes one cell (6 tets) and
// all load cases: it stages the cell's DOF box into LDS, lays the tets'
// coefficients out as columns (tet x load case x component), forms
// G = [D_1; D_2; D_3] X on the matrix cores (16x16x4 MFMA, FP32 or FP64), mixes
// the 9 derivative pairs with each tet's Q in place, forms Y = [D_1; D_2; D_3]^T H
// on the matrix cores, accumulates Y in an FP64 LDS box and writes the box to the
// cell's slot of the tile-box output (no global atomics).  The element energies
// x_e . y_e are summed on the way (p.Kp of the CG step).
#include "common.h"
#include "hp.h"
#include "internal.h"

#include <type_traits>

namespace chom {

using hp::Shape;

// Threads of an operator workgroup: 128 at order 3 (smaller per-cell work: more
// workgroups per CU hide the staging and barrier latency; 5.01 -> 4.65 ms per
// launch of 64 16^3 RVEs), 256 at order 4 (128: 12.6 -> 15.4 ms).
template <int P> constexpr int hp_threads() { return P == 3 ? 128 : 256; }

static inline int hp_grid(long long work, int bs, int cap = 16384) {
    long long g = (work + bs - 1) / bs;
    if (g < 1) g = 1;
    return (int)(g < cap ? g : cap);
}

// Lattice coordinates of local DOF q of tet e.
template <int P>
__device__ inline void hp_point(const Geo &G, long long e, int q, int &X, int &Y, int &Z) {
    const int n = G.n;
    const int t = (int)(e % 6);
    const long long cell = e / 6;
    const int ci = (int)(cell % n), cj = (int)((cell / n) % n), ck = (int)(cell / ((long long)n * n));
    const int *o = G.hoff + (t * Shape<P>::NE + q) * 3;
    X = P * ci + o[0];
    Y = P * cj + o[1];
    Z = P * ck + o[2];
}

// Q^{kl}_{cd} of one tet (k, l over grad lam_1..3), FP64.
template <int C>
__device__ inline void elem_Q(const double g[4][3], double vol, const double a[3], const double *m,
                              double Q[9][C][C]) {
    for (int l = 0; l < 3; ++l) {
        const double *w = g[l + 1];
        if constexpr (C == 3) {
            for (int d = 0; d < 3; ++d) {
                double G3[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
                for (int j = 0; j < 3; ++j) G3[d][j] = w[j];
                const double e[6] = {G3[0][0], G3[1][1], G3[2][2], 0.5 * (G3[0][1] + G3[1][0]),
                                     0.5 * (G3[1][2] + G3[2][1]), 0.5 * (G3[2][0] + G3[0][2])};
                double s[6];
                stress_ti<double>(e, a, m, s);
                const double sg[3][3] = {{s[0], s[3], s[5]}, {s[3], s[1], s[4]}, {s[5], s[4], s[2]}};
                for (int k = 0; k < 3; ++k) {
                    const double *gk = g[k + 1];
                    for (int c = 0; c < 3; ++c)
                        Q[k * 3 + l][c][d] = vol * (gk[0] * sg[c][0] + gk[1] * sg[c][1] + gk[2] * sg[c][2]);
                }
            }
        } else {
            double q[3];
            flux_ti<double>(w, a, m, q);
            for (int k = 0; k < 3; ++k) {
                const double *gk = g[k + 1];
                Q[k * 3 + l][0][0] = vol * (gk[0] * q[0] + gk[1] * q[1] + gk[2] * q[2]);
            }
        }
    }
}

// int grad(phi_q) dV of one tet.
template <int P>
__device__ inline void grad_integral(const Geo &G, const double g[4][3], double vol, int q, double w[3]) {
    constexpr int NE = Shape<P>::NE;
    for (int d = 0; d < 3; ++d)
        w[d] = vol * (G.hWd[q] * g[1][d] + G.hWd[NE + q] * g[2][d] + G.hWd[2 * NE + q] * g[3][d]);
}

// ------------------------------------------------------------------ constraint rows
template <int P>
__global__ void hp_rows_kernel(Geo G, double *rows) {
    constexpr int NE = Shape<P>::NE;
    const long long nt = 6LL * G.n * G.n * G.n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nt;
         e += (long long)gridDim.x * blockDim.x) {
        const int t = (int)(e % 6);
        double g[4][3], vol;
        GeoSel<double>::get(G, e, t, g, vol);
        for (int q = 0; q < NE; ++q) {
            int X, Y, Z;
            hp_point<P>(G, e, q, X, Y, Z);
            const long long idx = lat_index(G, X, Y, Z);
            double w[3];
            grad_integral<P>(G, g, vol, q, w);
            for (int d = 0; d < 3; ++d) atomicAdd(&rows[4 * idx + d], w[d]);
            atomicAdd(&rows[4 * idx + 3], vol * G.hW[q]);
        }
    }
}

hipError_t launch_rows_hp(const Geo &G, double *rows, hipStream_t s) {
    const long long nt = 6LL * G.n * G.n * G.n;
    if (G.p == 3) hp_rows_kernel<3><<<hp_grid(nt, 256), 256, 0, s>>>(G, rows);
    else hp_rows_kernel<4><<<hp_grid(nt, 256), 256, 0, s>>>(G, rows);
    return hipGetLastError();
}

// ------------------------------------------------------------------ block-Jacobi diagonal
template <int P, int C>
__global__ __launch_bounds__(256) void hp_diag_kernel(const Geo *geos, const Prob *probs, double *diag) {
    constexpr int NE = Shape<P>::NE;
    constexpr int MS = (C == 3) ? 6 : 1;
    const Prob &Pb = probs[blockIdx.y];
    const Geo &G = geos[Pb.geo];
    double *D = diag + Pb.doff * MS;
    const long long nt = 6LL * G.n * G.n * G.n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nt;
         e += (long long)gridDim.x * blockDim.x) {
        const int t = (int)(e % 6);
        double g[4][3], vol, a[3];
        int ph;
        GeoSel<double>::get(G, e, t, g, vol);
        GeoSel<double>::elem(G, e, a, ph);
        double Q[9][C][C];
        elem_Q<C>(g, vol, a, Pb.mat64[ph ? 1 : 0], Q);
        for (int q = 0; q < NE; ++q) {
            int X, Y, Z;
            hp_point<P>(G, e, q, X, Y, Z);
            if (dirichlet_boundary(G, X, Y, Z)) continue;
            const long long idx = lat_index(G, X, Y, Z);
            double B[C][C];
            for (int c = 0; c < C; ++c)
                for (int d = 0; d < C; ++d) {
                    double s = 0.0;
                    for (int kl = 0; kl < 9; ++kl) s += G.hSd[kl * NE + q] * Q[kl][c][d];
                    B[c][d] = s;
                }
            if constexpr (C == 3) {
                atomicAdd(&D[6 * idx + 0], B[0][0]);
                atomicAdd(&D[6 * idx + 1], B[1][1]);
                atomicAdd(&D[6 * idx + 2], B[2][2]);
                atomicAdd(&D[6 * idx + 3], 0.5 * (B[0][1] + B[1][0]));
                atomicAdd(&D[6 * idx + 4], 0.5 * (B[1][2] + B[2][1]));
                atomicAdd(&D[6 * idx + 5], 0.5 * (B[0][2] + B[2][0]));
            } else {
                atomicAdd(&D[idx], B[0][0]);
            }
        }
    }
}

template <int C>
hipError_t launch_diag_hp(const Launch &L, double *diag, hipStream_t s) {
    dim3 grid(hp_grid(L.max_tets, 256, 2048), L.nprob);
    if (L.order == 3) hp_diag_kernel<3, C><<<grid, 256, 0, s>>>(L.geos, L.probs, diag);
    else hp_diag_kernel<4, C><<<grid, 256, 0, s>>>(L.geos, L.probs, diag);
    return hipGetLastError();
}
template hipError_t launch_diag_hp<3>(const Launch &, double *, hipStream_t);
template hipError_t launch_diag_hp<1>(const Launch &, double *, hipStream_t);

// ------------------------------------------------------------------ load vectors
// Same definitions as the order-2 kernel: b = -int grad(phi) : C eps_k and the
// linear-field energy.
template <int P, int C, int R>
__global__ void hp_rhs_kernel(const Geo *geos, const Prob *probs, double *b, ColState *cols) {
    constexpr int NE = Shape<P>::NE;
    const int prob = blockIdx.y;
    const Prob &Pb = probs[prob];
    const Geo &G = geos[Pb.geo];
    double *bp = b + Pb.voff;
    const long long nt = 6LL * G.n * G.n * G.n;
    double eref[R];
    for (int k = 0; k < R; ++k) eref[k] = 0.0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nt;
         e += (long long)gridDim.x * blockDim.x) {
        const int t = (int)(e % 6);
        double g[4][3], vol, a[3];
        int ph;
        GeoSel<double>::get(G, e, t, g, vol);
        GeoSel<double>::elem(G, e, a, ph);
        const double *m = Pb.mat64[ph ? 1 : 0];
        for (int k = 0; k < R; ++k) {
            double sig[3][3];
            if constexpr (C == 3) {
                double eps[6] = {0, 0, 0, 0, 0, 0};
                if (k < 3) eps[k] = 1.0; else eps[k] = 0.5;
                double s[6];
                stress_ti<double>(eps, a, m, s);
                sig[0][0] = s[0]; sig[1][1] = s[1]; sig[2][2] = s[2];
                sig[0][1] = sig[1][0] = s[3];
                sig[1][2] = sig[2][1] = s[4];
                sig[2][0] = sig[0][2] = s[5];
                eref[k] += vol * s[k];
            } else {
                double gk[3] = {0, 0, 0};
                gk[k] = 1.0;
                double q[3];
                flux_ti<double>(gk, a, m, q);
                sig[0][0] = q[0]; sig[0][1] = q[1]; sig[0][2] = q[2];
                eref[k] += vol * q[k];
            }
            for (int q = 0; q < NE; ++q) {
                int X, Y, Z;
                hp_point<P>(G, e, q, X, Y, Z);
                if (dirichlet_boundary(G, X, Y, Z)) continue;
                double w[3];
                grad_integral<P>(G, g, vol, q, w);
                const long long idx = lat_index(G, X, Y, Z);
                for (int c = 0; c < C; ++c)
                    atomicAdd(&bp[(k * G.npts + idx) * C + c], -(sig[c][0] * w[0] + sig[c][1] * w[1] + sig[c][2] * w[2]));
            }
        }
    }
    __shared__ double red[R][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < R; ++k) {
        const double v = wave_sum(eref[k]);
        if (lane == 0) red[k][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < R) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[threadIdx.x][w];
        atomicAdd(&cols[prob * R + threadIdx.x].eref, s);
    }
}

template <int C, int R>
hipError_t launch_rhs_hp(const Launch &L, double *b, ColState *cols, hipStream_t s) {
    dim3 grid(hp_grid(L.max_tets, 256, 2048), L.nprob);
    if (L.order == 3) hp_rhs_kernel<3, C, R><<<grid, 256, 0, s>>>(L.geos, L.probs, b, cols);
    else hp_rhs_kernel<4, C, R><<<grid, 256, 0, s>>>(L.geos, L.probs, b, cols);
    return hipGetLastError();
}
template hipError_t launch_rhs_hp<3, 6>(const Launch &, double *, ColState *, hipStream_t);
template hipError_t launch_rhs_hp<1, 3>(const Launch &, double *, ColState *, hipStream_t);

// ------------------------------------------------------------------ homogenisation average
// Partial sums per workgroup of sum_e C_e (eps_k |e| + int sym grad(u~_k)), as the
// order-2 kernel (Eq. macro_stress, Eq. Eq_C_stress; Eq. eq_homo_flux).
template <int P, int C, int R>
__global__ __launch_bounds__(256) void hp_average_kernel(const Geo *geos, const Prob *probs, const double *x, double *partial) {
    constexpr int NE = Shape<P>::NE;
    constexpr int NC = (C == 3) ? 6 : 3;
    const int prob = blockIdx.y;
    const Prob &Pb = probs[prob];
    const Geo &G = geos[Pb.geo];
    const double *xp = x + Pb.voff;
    const long long nt = 6LL * G.n * G.n * G.n;
    double acc[R * NC];
    for (int k = 0; k < R * NC; ++k) acc[k] = 0.0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nt;
         e += (long long)gridDim.x * blockDim.x) {
        const int t = (int)(e % 6);
        double g[4][3], vol, a[3];
        int ph;
        GeoSel<double>::get(G, e, t, g, vol);
        GeoSel<double>::elem(G, e, a, ph);
        const double *m = Pb.mat64[ph ? 1 : 0];
        for (int r = 0; r < R; ++r) {
            double H[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            for (int q = 0; q < NE; ++q) {
                int X, Y, Z;
                hp_point<P>(G, e, q, X, Y, Z);
                const long long idx = lat_index(G, X, Y, Z);
                double w[3];
                grad_integral<P>(G, g, vol, q, w);
                for (int c = 0; c < C; ++c) {
                    const double u = xp[(r * G.npts + idx) * C + c];
                    for (int d = 0; d < 3; ++d) H[c][d] += u * w[d];
                }
            }
            if constexpr (C == 3) {
                double eps[6] = {H[0][0], H[1][1], H[2][2], 0.5 * (H[0][1] + H[1][0]),
                                 0.5 * (H[1][2] + H[2][1]), 0.5 * (H[2][0] + H[0][2])};
                if (r < 3) eps[r] += vol; else eps[r] += 0.5 * vol;
                double s[6];
                stress_ti<double>(eps, a, m, s);
                for (int k = 0; k < 6; ++k) acc[r * NC + k] += s[k];
            } else {
                double gr[3] = {H[0][0], H[0][1], H[0][2]};
                gr[r] += vol;
                double q[3];
                flux_ti<double>(gr, a, m, q);
                for (int k = 0; k < 3; ++k) acc[r * NC + k] += q[k];
            }
        }
    }
    __shared__ double red[R * NC][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < R * NC; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) red[k][wv] = v;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < R * NC; k += blockDim.x) {
        double s = 0.0;
        for (int w2 = 0; w2 < (int)(blockDim.x >> 6); ++w2) s += red[k][w2];
        partial[((long long)prob * gridDim.x + blockIdx.x) * R * NC + k] = s;
    }
}

template <int C, int R>
hipError_t launch_average_partial_hp(const Launch &L, const double *x64, double *partial, int nwg, hipStream_t s) {
    dim3 grid(nwg, L.nprob);
    if (L.order == 3) hp_average_kernel<3, C, R><<<grid, 256, 0, s>>>(L.geos, L.probs, x64, partial);
    else hp_average_kernel<4, C, R><<<grid, 256, 0, s>>>(L.geos, L.probs, x64, partial);
    return hipGetLastError();
}
template hipError_t launch_average_partial_hp<3, 6>(const Launch &, const double *, double *, int, hipStream_t);
template hipError_t launch_average_partial_hp<1, 3>(const Launch &, const double *, double *, int, hipStream_t);

// ------------------------------------------------------------------ operator
// 16x16x4 matrix-core products.  Lane l supplies A[l & 15][l >> 4] and
// B[l >> 4][l & 15]; result register q of lane l holds C[row(l >> 4, q)][l & 15],
// with row = 4 (l >> 4) + q for FP32 and (l >> 4) + 4 q for FP64 (measured).
template <typename T> struct Mfma;
template <> struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __device__ static inline int row(int lk, int q) { return 4 * lk + q; }
    __device__ static inline v4 op(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static inline const float *DA(const Geo &G) { return G.hDA32; }
    __device__ static inline const float *DB(const Geo &G) { return G.hDB32; }
};
template <> struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __device__ static inline int row(int lk, int q) { return lk + 4 * q; }
    __device__ static inline v4 op(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static inline const double *DA(const Geo &G) { return G.hDA64; }
    __device__ static inline const double *DB(const Geo &G) { return G.hDB64; }
};

// ------------------------------------------------------------------ element factors
// Q_e of every tet of every problem, packed: upper triangle (row-major) of the
// symmetric (3C) x (3C) matrix with index (k, c) = k C + c (45 numbers per element for
// the mechanics, 6 for a scalar field), FP64 master and FP32 copy.
template <int C>
__global__ __launch_bounds__(256) void hp_factor_kernel(const Geo *geos, const Prob *probs, double *ef64, float *ef32) {
    constexpr int NQ = (3 * C) * (3 * C + 1) / 2;
    const Prob &Pb = probs[blockIdx.y];
    const Geo &G = geos[Pb.geo];
    const long long nt = 6LL * G.n * G.n * G.n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nt;
         e += (long long)gridDim.x * blockDim.x) {
        const int t = (int)(e % 6);
        double g[4][3], vol, a[3];
        int ph;
        GeoSel<double>::get(G, e, t, g, vol);
        GeoSel<double>::elem(G, e, a, ph);
        double Q[9][C][C];
        elem_Q<C>(g, vol, a, Pb.mat64[ph ? 1 : 0], Q);
        double *o64 = ef64 + Pb.eoff + e * NQ;
        float *o32 = ef32 + Pb.eoff + e * NQ;
        int u = 0;
        for (int I = 0; I < 3 * C; ++I)
            for (int J = I; J < 3 * C; ++J) {
                const int k = I / C, c = I % C, l = J / C, d = J % C;
                const double v = Q[k * 3 + l][c][d];
                o64[u] = v;
                o32[u] = (float)v;
                ++u;
            }
    }
}

template <int C>
hipError_t launch_factors_hp(const Launch &L, double *ef64, float *ef32, hipStream_t s) {
    dim3 grid(hp_grid(L.max_tets, 256, 4096), L.nprob);
    hp_factor_kernel<C><<<grid, 256, 0, s>>>(L.geos, L.probs, ef64, ef32);
    return hipGetLastError();
}
template hipError_t launch_factors_hp<3>(const Launch &, double *, float *, hipStream_t);
template hipError_t launch_factors_hp<1>(const Launch &, double *, float *, hipStream_t);

// ------------------------------------------------------------------ operator
// One workgroup: one cell (its 6 tets), all R load cases.  The cell's (p+1)^3 DOF
// box is staged from HBM once; the element results accumulate in an FP64 LDS box
// that is written, contiguous, to the cell's slot of the tile-box output
// (consumers sum the copies of points shared by neighbouring cells).
template <typename T, int P, int C, int R>
__global__ __launch_bounds__(hp_threads<P>()) void hp_op_kernel(const Geo *geos, const Prob *probs, int max_tiles,
                                                          const T *__restrict__ x, T *__restrict__ y,
                                                          const T *__restrict__ ef, double *acc_pq,
                                                          const int *prob_active) {
    using Sh = Shape<P>;
    constexpr int NE = Sh::NE, M = Sh::M, MA = Sh::MA, KA = Sh::KA, MB = Sh::MB, KB = Sh::KB;
    constexpr int NQ = (3 * C) * (3 * C + 1) / 2;
    constexpr int EB = 6;
    constexpr int RC = R * C;
    constexpr int B1 = P + 1, BP = B1 * B1 * B1;
    constexpr int NC = EB * RC;              // columns: tet x load case x component
    constexpr int NT = (NC + 15) / 16;
    constexpr int NCP = NT * 16;
    constexpr int HP_THREADS = hp_threads<P>();
    constexpr int NW = HP_THREADS / 64;
    using V4 = typename Mfma<T>::v4;
    // LDS shared by phases: X (xs) is dead once G is formed, so the output box
    // yb takes its place (cleared after the G product; the element energies are
    // formed from the box at write-back).  At order 4 the staged box xb is also
    // dead once X is built and G/H (gs) take its place (x for the energies is
    // then read again from memory): 50 instead of 75 KB, three workgroups per CU.
    constexpr bool XB_IN_GS = P >= 4;
    constexpr int GSB = (int)(MA * NCP * sizeof(T)), XBB = (int)(BP * RC * sizeof(T));
    constexpr int U1 = XB_IN_GS ? (XBB > GSB ? XBB : GSB) : GSB;
    constexpr int U2 = (int)(KA * NCP * sizeof(T) > BP * RC * sizeof(double) ? KA * NCP * sizeof(T)
                                                                           : BP * RC * sizeof(double));
    __shared__ __align__(16) unsigned char u1[U1];
    __shared__ __align__(16) unsigned char u2[U2];
    __shared__ __align__(16) unsigned char u0[XB_IN_GS ? 16 : XBB];
    T *const xb = XB_IN_GS ? (T *)u1 : (T *)u0;
    T(*const gs)[NCP] = (T(*)[NCP])u1;
    T(*const xs)[NCP] = (T(*)[NCP])u2;
    double *const yb = (double *)u2;
    __shared__ T qs[EB][3 * C][3 * C];
    __shared__ int bidx[EB][NE];
    __shared__ double red[R][NW];
    const int prob = blockIdx.y;
    const int cell = blockIdx.x;
    const Prob &Pb = probs[prob];
    const Geo &G = geos[Pb.geo];
    const int n = G.n;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (cell >= n * n * n || (prob_active != nullptr && prob_active[prob] == 0)) return;
    const int ci = cell % n, cj = (cell / n) % n, ck = cell / (n * n);
    // ---- stage the DOF box, clear the output box, box index of every local DOF, factors
    const T *xp = x + Pb.voff;
    for (int i = tid; i < BP * RC; i += HP_THREADS) {
        const int pt = i / RC, v = i - (i / RC) * RC;
        const int r = v / C, c = v - (v / C) * C;
        const int bx = pt % B1, by = (pt / B1) % B1, bz = pt / (B1 * B1);
        const long long idx = lat_index(G, P * ci + bx, P * cj + by, P * ck + bz);
        xb[i] = xp[((long long)r * G.npts + idx) * C + c];
    }
    for (int i = tid; i < EB * NE; i += HP_THREADS) {
        const int e = i / NE, q = i - (i / NE) * NE;
        const int *o = G.hoff + (e * NE + q) * 3;
        bidx[e][q] = o[0] + B1 * (o[1] + B1 * o[2]);
    }
    for (int i = tid; i < EB * NQ; i += HP_THREADS) {
        const int e = i / NQ, u = i - (i / NQ) * NQ;
        int I = 0, rem = u;
        while (rem >= 3 * C - I) {
            rem -= 3 * C - I;
            ++I;
        }
        const int J = I + rem;
        const T v = ef[Pb.eoff + ((long long)cell * 6 + e) * NQ + u];
        qs[e][I][J] = v;
        qs[e][J][I] = v;
    }
    __syncthreads();
    // ---- X [KA][NCP]: column (tet * R + load case) * C + component
    for (int i = tid; i < KA * NCP; i += HP_THREADS) {
        const int j = i / NCP, col = i - (i / NCP) * NCP;
        T v = T(0);
        if (j < NE && col < NC) {
            const int e = col / RC, rem = col - (col / RC) * RC;
            v = xb[bidx[e][j] * RC + rem];
        }
        xs[j][col] = v;
    }
    __syncthreads();
    // ---- G = DA X on the matrix cores: each wave keeps all of DA's fragments in
    // registers and sweeps its column tiles, reusing each X fragment for all row tiles
    const T *DA = Mfma<T>::DA(G);
    const T *DB = Mfma<T>::DB(G);
    const int lr = lane & 15, lk = lane >> 4;
    {
        constexpr int MT = MA / 16, KS = KA / 4;
        T af[MT][KS];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) af[mt][ks] = DA[(mt * 16 + lr) * KA + ks * 4 + lk];
        for (int ct = wave; ct < NT; ct += NW) {
            V4 acc[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt] = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const T b = xs[ks * 4 + lk][ct * 16 + lr];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt] = Mfma<T>::op(af[mt][ks], b, acc[mt]);
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int q = 0; q < 4; ++q) gs[mt * 16 + Mfma<T>::row(lk, q)][ct * 16 + lr] = acc[mt][q];
        }
    }
    __syncthreads();
    for (int i = tid; i < BP * RC; i += HP_THREADS) yb[i] = 0.0;   // X is dead: its space holds the output box
    // ---- H = sum_l Q^{kl} G_l, in place (rows k*M + a)
    for (int i = tid; i < M * EB * R; i += HP_THREADS) {
        const int a = i % M, er = i / M;
        const int e = er / R;
        const int col0 = er * C;
        T gv[3 * C];
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int d = 0; d < C; ++d) gv[l * C + d] = gs[l * M + a][col0 + d];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                T h = T(0);
#pragma unroll
                for (int J = 0; J < 3 * C; ++J) h += qs[e][k * C + c][J] * gv[J];
                gs[k * M + a][col0 + c] = h;
            }
    }
    __syncthreads();
    // ---- Y = DB H on the matrix cores; accumulate into the LDS box, element energies
    double pq[R];
#pragma unroll
    for (int r = 0; r < R; ++r) pq[r] = 0.0;
    {
        constexpr int MT = MB / 16, KS = KB / 4;
        T bf[MT][KS];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) bf[mt][ks] = DB[(mt * 16 + lr) * KB + ks * 4 + lk];
        for (int ct = wave; ct < NT; ct += NW) {
            V4 acc[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) acc[mt] = V4{T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const T b = gs[ks * 4 + lk][ct * 16 + lr];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt] = Mfma<T>::op(bf[mt][ks], b, acc[mt]);
            }
            const int col = ct * 16 + lr;
            if (col >= NC) continue;
            const int e = col / RC, rem = col - (col / RC) * RC;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = mt * 16 + Mfma<T>::row(lk, q);
                    if (i >= NE) continue;
                    atomicAdd(&yb[bidx[e][i] * RC + rem], (double)acc[mt][q]);
                }
        }
    }
    __syncthreads();
    // ---- write the cell's box (contiguous); the cell's energies x_e . K_e x_e
    // summed over its tets are x . y over its box (x read again, cached)
    T *yt = y + Pb.qoff + (long long)cell * BP * RC;
    for (int i = tid; i < BP * RC; i += HP_THREADS) {   // load-case major: i = (r * BP + pt) * C + c
        const int r = i / (BP * C), rem = i - r * (BP * C);
        const int pt = rem / C, c = rem - (rem / C) * C;
        const double v = yb[pt * RC + r * C + c];
        yt[i] = (T)v;
        double xv;
        if constexpr (XB_IN_GS) {
            const int bx = pt % B1, by = (pt / B1) % B1, bz = pt / (B1 * B1);
            const long long idx = lat_index(G, P * ci + bx, P * cj + by, P * ck + bz);
            xv = (double)xp[((long long)r * G.npts + idx) * C + c];
        } else {
            xv = (double)xb[pt * RC + r * C + c];
        }
        const double en = xv * v;
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
            if (rr == r) pq[rr] += en;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double sm = wave_sum(pq[r]);
        if (lane == 0) red[r][wave] = sm;
    }
    __syncthreads();
    if (tid < R) {
        double sm = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) sm += red[tid][w];
        unsafeAtomicAdd(&acc_pq[((long long)prob * R + tid) * ACC_STRIPES + (cell & (ACC_STRIPES - 1))], sm);
    }
}

template <typename T, int P, int C, int R>
static hipError_t launch_hp(const Launch &L, int nprob, const T *x, T *y, double *acc_pq, const int *prob_active,
                            hipStream_t s) {
    dim3 grid(L.max_tiles, nprob);
    const T *ef = std::is_same<T, double>::value ? (const T *)L.ef64 : (const T *)L.ef32;
    hp_op_kernel<T, P, C, R><<<grid, hp_threads<P>(), 0, s>>>(L.geos, L.probs, L.max_tiles, x, y, ef, acc_pq,
                                                         prob_active);
    return hipGetLastError();
}

template <typename T, int C, int R>
hipError_t launch_operator_hp(const Launch &L, int nprob, int /*rg*/, const T *x, T *y, double *acc_pq,
                              const int *prob_active, hipStream_t s) {
    if (L.order == 3) return launch_hp<T, 3, C, R>(L, nprob, x, y, acc_pq, prob_active, s);
    return launch_hp<T, 4, C, R>(L, nprob, x, y, acc_pq, prob_active, s);
}

template hipError_t launch_operator_hp<double, 3, 6>(const Launch &, int, int, const double *, double *, double *, const int *, hipStream_t);
template hipError_t launch_operator_hp<float, 3, 6>(const Launch &, int, int, const float *, float *, double *, const int *, hipStream_t);
template hipError_t launch_operator_hp<double, 1, 3>(const Launch &, int, int, const double *, double *, double *, const int *, hipStream_t);
template hipError_t launch_operator_hp<float, 1, 3>(const Launch &, int, int, const float *, float *, double *, const int *, hipStream_t);

}  // namespace chom
