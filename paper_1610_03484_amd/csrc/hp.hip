// Orders p = 3, 4: setup kernels and the element-batched operator.
//
// K_e of Sec. 2 (Eq. eq_RVE_disc_Eqs; Eq. eq_RVE_disc_Eqs_field for the scalar
// fields) for the order-p hierarchic space, applied as
//   y_e = sum_k D_k^T [ sum_l Q_e^{kl} (D_l x_e) ],
//   Q_e^{kl}_{cd} = |e| sum_mn (grad lam_k)_m C_{cmdn} (grad lam_l)_n   (k, l = 1..3),
// where D_k are the order's derivative tables in a mass-orthonormal basis of
// P_{p-1} (shared by every tet).  A workgroup takes 16 tets and a group of load
// cases: it gathers their coefficients into LDS (columns = tet x load case x
// component), forms G = [D_1; D_2; D_3] X on the matrix cores (16x16x4 MFMA,
// FP32 or FP64), mixes the 9 derivative pairs with each tet's Q in place, forms
// Y = [D_1; D_2; D_3]^T H on the matrix cores, and adds Y into the output vector
// with global atomics (the output is cleared first).  The element energies
// x_e . y_e are summed on the way (p.Kp of the CG step).
#include "common.h"
#include "hp.h"
#include "internal.h"

namespace chom {

using hp::Shape;

constexpr int HP_EB = hp::OP_TETS;
constexpr int HP_THREADS = 256;

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
__global__ void hp_diag_kernel(const Geo *geos, const Prob *probs, double *diag) {
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
__global__ void hp_average_kernel(const Geo *geos, const Prob *probs, const double *x, double *partial) {
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

template <typename T, int P, int C, int R, int RG>
__global__ __launch_bounds__(HP_THREADS) void hp_op_kernel(const Geo *geos, const Prob *probs, int max_batches,
                                                          const T *__restrict__ x, T *__restrict__ y,
                                                          double *partial_pq, const int *prob_active) {
    using Sh = Shape<P>;
    constexpr int NE = Sh::NE, M = Sh::M, MA = Sh::MA, KA = Sh::KA, MB = Sh::MB, KB = Sh::KB;
    constexpr int NG = R / RG;
    constexpr int NC = HP_EB * RG * C;       // columns: tet x load case x component
    constexpr int NT = (NC + 15) / 16;
    constexpr int NCP = NT * 16;
    constexpr int NW = HP_THREADS / 64;
    using V4 = typename Mfma<T>::v4;
    __shared__ T xs[KA][NCP];
    __shared__ T gs[MA][NCP];
    __shared__ T qs[HP_EB][9][C][C];
    __shared__ long long pidx[HP_EB][NE];
    __shared__ double red[RG][NW];
    const int prob = blockIdx.y;
    const int batch = blockIdx.x / NG, grp = blockIdx.x - (blockIdx.x / NG) * NG;
    const Prob &Pb = probs[prob];
    const Geo &G = geos[Pb.geo];
    const long long nt = 6LL * G.n * G.n * G.n;
    const long long e0 = (long long)batch * HP_EB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (e0 >= nt || (prob_active != nullptr && prob_active[prob] == 0)) {
        if (tid < RG) partial_pq[((long long)prob * R + grp * RG + tid) * max_batches + batch] = 0.0;
        return;
    }
    // ---- per-tet data: Q and the lattice index of every local DOF
    if (tid < HP_EB) {
        const long long e = e0 + tid;
        if (e < nt) {
            const int t = (int)(e % 6);
            double g[4][3], vol, a[3];
            int ph;
            GeoSel<double>::get(G, e, t, g, vol);
            GeoSel<double>::elem(G, e, a, ph);
            double Q[9][C][C];
            elem_Q<C>(g, vol, a, Pb.mat64[ph ? 1 : 0], Q);
            for (int kl = 0; kl < 9; ++kl)
                for (int c = 0; c < C; ++c)
                    for (int d = 0; d < C; ++d) qs[tid][kl][c][d] = (T)Q[kl][c][d];
            for (int q = 0; q < NE; ++q) {
                int X, Y, Z;
                hp_point<P>(G, e, q, X, Y, Z);
                pidx[tid][q] = lat_index(G, X, Y, Z);
            }
        } else {
            for (int kl = 0; kl < 9; ++kl)
                for (int c = 0; c < C; ++c)
                    for (int d = 0; d < C; ++d) qs[tid][kl][c][d] = T(0);
            for (int q = 0; q < NE; ++q) pidx[tid][q] = -1;
        }
    }
    __syncthreads();
    // ---- gather X [KA][NCP]: column (tet * RG + load case) * C + component
    const T *xp = x + Pb.voff;
    for (int i = tid; i < KA * NCP; i += HP_THREADS) {
        const int j = i / NCP, col = i - (i / NCP) * NCP;
        T v = T(0);
        if (j < NE && col < NC) {
            const int e = col / (RG * C), rem = col - (col / (RG * C)) * (RG * C);
            const int r = rem / C, d = rem - (rem / C) * C;
            const long long pt = pidx[e][j];
            if (pt >= 0) v = xp[((long long)(grp * RG + r) * G.npts + pt) * C + d];
        }
        xs[j][col] = v;
    }
    __syncthreads();
    // ---- G = DA X on the matrix cores
    const T *DA = Mfma<T>::DA(G);
    const T *DB = Mfma<T>::DB(G);
    const int lr = lane & 15, lk = lane >> 4;
    for (int tile = wave; tile < (MA / 16) * NT; tile += NW) {
        const int mt = tile / NT, ct = tile - (tile / NT) * NT;
        V4 acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int k0 = 0; k0 < KA; k0 += 4)
            acc = Mfma<T>::op(DA[(mt * 16 + lr) * KA + k0 + lk], xs[k0 + lk][ct * 16 + lr], acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) gs[mt * 16 + Mfma<T>::row(lk, q)][ct * 16 + lr] = acc[q];
    }
    __syncthreads();
    // ---- H = sum_l Q^{kl} G_l, in place (rows k*M + a)
    for (int i = tid; i < M * HP_EB * RG; i += HP_THREADS) {
        const int a = i % M, er = i / M;
        const int e = er / RG, r = er - (er / RG) * RG;
        const int col0 = (e * RG + r) * C;
        T gv[3][C];
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int d = 0; d < C; ++d) gv[l][d] = gs[l * M + a][col0 + d];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                T h = T(0);
#pragma unroll
                for (int l = 0; l < 3; ++l)
#pragma unroll
                    for (int d = 0; d < C; ++d) h += qs[e][k * 3 + l][c][d] * gv[l][d];
                gs[k * M + a][col0 + c] = h;
            }
    }
    __syncthreads();
    // ---- Y = DB H on the matrix cores; add into y, element energies
    T *yp = y + Pb.qoff;
    double pq[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) pq[r] = 0.0;
    for (int tile = wave; tile < (MB / 16) * NT; tile += NW) {
        const int mt = tile / NT, ct = tile - (tile / NT) * NT;
        V4 acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int k0 = 0; k0 < KB; k0 += 4)
            acc = Mfma<T>::op(DB[(mt * 16 + lr) * KB + k0 + lk], gs[k0 + lk][ct * 16 + lr], acc);
        const int col = ct * 16 + lr;
        if (col < NC) {
            const int e = col / (RG * C), rem = col - (col / (RG * C)) * (RG * C);
            const int r = rem / C, d = rem - (rem / C) * C;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = mt * 16 + Mfma<T>::row(lk, q);
                if (i >= NE) continue;
                const long long pt = pidx[e][i];
                if (pt < 0) continue;
                atomicAdd(&yp[((long long)(grp * RG + r) * G.npts + pt) * C + d], acc[q]);
                const double en = (double)xs[i][col] * (double)acc[q];
#pragma unroll
                for (int rr = 0; rr < RG; ++rr)
                    if (rr == r) pq[rr] += en;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RG; ++r) {
        const double s = wave_sum(pq[r]);
        if (lane == 0) red[r][wave] = s;
    }
    __syncthreads();
    if (tid < RG) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += red[tid][w];
        partial_pq[((long long)prob * R + grp * RG + tid) * max_batches + batch] = s;
    }
}

template <typename T>
__global__ void hp_clear_kernel(T *y, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        y[i] = T(0);
}

template <typename T, int P, int C, int R, int RG>
static hipError_t launch_hp_rg(const Launch &L, int nprob, const T *x, T *y, double *partial_pq,
                               const int *prob_active, hipStream_t s) {
    dim3 grid(L.max_tiles * (R / RG), nprob);
    hp_op_kernel<T, P, C, R, RG><<<grid, HP_THREADS, 0, s>>>(L.geos, L.probs, L.max_tiles, x, y, partial_pq,
                                                              prob_active);
    return hipGetLastError();
}

template <typename T, int C, int R>
hipError_t launch_operator_hp(const Launch &L, int nprob, int rg, const T *x, T *y, double *partial_pq,
                              const int *prob_active, hipStream_t s) {
    hp_clear_kernel<T><<<hp_grid(L.total_q, 256), 256, 0, s>>>(y, L.total_q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if constexpr (C == 3) {
        if (rg == 1) {
            if (L.order == 3) return launch_hp_rg<T, 3, C, R, 1>(L, nprob, x, y, partial_pq, prob_active, s);
            return launch_hp_rg<T, 4, C, R, 1>(L, nprob, x, y, partial_pq, prob_active, s);
        }
        if (L.order == 3) return launch_hp_rg<T, 3, C, R, 2>(L, nprob, x, y, partial_pq, prob_active, s);
        return launch_hp_rg<T, 4, C, R, 2>(L, nprob, x, y, partial_pq, prob_active, s);
    } else {
        if (L.order == 3) return launch_hp_rg<T, 3, C, R, 3>(L, nprob, x, y, partial_pq, prob_active, s);
        return launch_hp_rg<T, 4, C, R, 3>(L, nprob, x, y, partial_pq, prob_active, s);
    }
}

template hipError_t launch_operator_hp<double, 3, 6>(const Launch &, int, int, const double *, double *, double *, const int *, hipStream_t);
template hipError_t launch_operator_hp<float, 3, 6>(const Launch &, int, int, const float *, float *, double *, const int *, hipStream_t);
template hipError_t launch_operator_hp<double, 1, 3>(const Launch &, int, int, const double *, double *, double *, const int *, hipStream_t);
template hipError_t launch_operator_hp<float, 1, 3>(const Launch &, int, int, const float *, float *, double *, const int *, hipStream_t);

}  // namespace chom
