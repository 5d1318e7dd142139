// Preconditioned conjugate gradients on the constrained RVE system, many
// problems and load cases at once.
//
// The paper solves the saddle-point system of Eq. eq_RVE_disc_Eqs with a
// direct factorisation; it notes that projection is an equivalent route (Sec.
// 2, after Eq. eq_X_mech).  Here the fluctuation is found by CG on ker(C): with
// the block-Jacobi preconditioner M and the constraint rows C (periodic: the
// mean of each component; uniform traction: the surface moments and the mean),
// the preconditioner is z = P M^-1 r with the M-oblique projector
//   P M^-1 = M^-1 - M^-1 C^T (C M^-1 C^T)^-1 C M^-1,
// which maps into ker(C) and annihilates range(C^T), so the unprojected
// residual can be carried.  r.z, its pieces and p.Kp are accumulated in FP64
// whatever the vector precision.
//
// Partial-sum layout per (problem, block, load case): [r.z0, r.r, C z0 (C*NR)].
#include "common.h"
#include "internal.h"

namespace chom {

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

template <int N>
__device__ inline void block_reduce_store(double (&acc)[N], double *dst) {
    __shared__ double red[N][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) red[k][wv] = s;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[k][w];
        dst[k] = s;
    }
}

__device__ inline void point_range(long long npts, long long &p0, long long &p1) {
    const long long per = (npts + gridDim.x - 1) / gridDim.x;
    p0 = blockIdx.x * per;
    p1 = p0 + per < npts ? p0 + per : npts;
}

// Vector kernels: one workgroup = R waves, wave w handles load case w for 64
// consecutive lattice points at a time (grid-stride over point blocks).  Each
// wave reduces its own column, so the partial sums need no block barrier.
// Partial layout (k-major): partial[((prob * R + w) * REC + k) * nwg + block].
__device__ inline void wave_partials(const double *acc, int REC, double *partial, int prob, int R, int w) {
    const int lane = threadIdx.x & 63;
    for (int k = 0; k < REC; ++k) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) partial[(((long long)prob * R + w) * REC + k) * gridDim.x + blockIdx.x] = s;
    }
}

// r = b, x = 0, z0 = M^-1 r; partial sums.  WRITE = false: only the sums.
template <typename T, int C, int R, int NR, bool WRITE>
__global__ __launch_bounds__(64 * R) void cg_init_kernel(Geo G, long long vpp, const T *b, T *x, T *r,
                                                         T *z, const T *minv, double *partial) {
    constexpr int MS = (C == 3) ? 6 : 1;
    constexpr int REC = 2 + C * NR;
    constexpr int RF = (NR == 1) ? 3 : 0;
    const int prob = blockIdx.y;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long base = (long long)prob * vpp;
    const T *Mp = minv + (long long)prob * G.npts * MS;
    double acc[REC];
#pragma unroll
    for (int k = 0; k < REC; ++k) acc[k] = 0.0;
    const long long nblk = (G.npts + 63) / 64;
    for (long long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const long long pt = blk * 64 + lane;
        if (pt >= G.npts) continue;
        T Mi[MS];
#pragma unroll
        for (int k = 0; k < MS; ++k) Mi[k] = Mp[pt * MS + k];
        double row[4] = {0, 0, 0, 0};
#pragma unroll
        for (int a = 0; a < NR; ++a) row[a] = G.rows[4 * pt + RF + a];
        const long long o = base + (pt * R + w) * C;
        T rv[C], zv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) rv[c] = b[o + c];
        minv_apply<T, C>(Mi, rv, zv);
        if constexpr (WRITE) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                r[o + c] = rv[c];
                x[o + c] = T(0);
                z[o + c] = zv[c];
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            acc[0] += (double)rv[c] * (double)zv[c];
            acc[1] += (double)rv[c] * (double)rv[c];
#pragma unroll
            for (int a = 0; a < NR; ++a) acc[2 + c * NR + a] += row[a] * (double)zv[c];
        }
    }
    wave_partials(acc, REC, partial, prob, R, w);
}

// z = z0 - M^-1 C^T y ; r = r - C^T y ; p = z + beta p.
template <typename T, int C, int R, int NR>
__global__ __launch_bounds__(64 * R) void cg_dir_kernel(Geo G, long long vpp, T *r, const T *z, T *p, T *q,
                                                        const T *minv, const double *ycoef,
                                                        const ColState *cols, const int *prob_active) {
    constexpr int MS = (C == 3) ? 6 : 1;
    constexpr int S = C * NR;
    constexpr int RF = (NR == 1) ? 3 : 0;
    const int prob = blockIdx.y;
    if (prob_active[prob] == 0) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double beta = cols[prob * R + w].beta;
    double yv[S > 0 ? S : 1];
#pragma unroll
    for (int k = 0; k < S; ++k) yv[k] = ycoef[((long long)prob * R + w) * S + k];
    const long long base = (long long)prob * vpp;
    const T *Mp = minv + (long long)prob * G.npts * MS;
    const long long nblk = (G.npts + 63) / 64;
    for (long long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const long long pt = blk * 64 + lane;
        if (pt >= G.npts) continue;
        const long long o = base + (pt * R + w) * C;
        T zv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) zv[c] = z[o + c];
        if constexpr (NR > 0) {
            // projection correction M^-1 C^T y evaluated in FP64
            double Md[MS], ct[C], corr[C], row[4] = {0, 0, 0, 0};
#pragma unroll
            for (int k = 0; k < MS; ++k) Md[k] = (double)Mp[pt * MS + k];
#pragma unroll
            for (int a = 0; a < NR; ++a) row[a] = G.rows[4 * pt + RF + a];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                ct[c] = 0.0;
#pragma unroll
                for (int a = 0; a < NR; ++a) ct[c] += row[a] * yv[c * NR + a];
            }
            minv_apply<double, C>(Md, ct, corr);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                zv[c] = (T)((double)zv[c] - corr[c]);
                // residual projected the same way (adjoint projector), so the
                // multiplier forces do not pile up in r and r.z stays accurate
                r[o + c] = (T)((double)r[o + c] - ct[c]);
            }
        }
        if (beta == 0.0) {   // first step (p not yet defined) or finished column
#pragma unroll
            for (int c = 0; c < C; ++c) p[o + c] = zv[c];
        } else {
            const T bt = (T)beta;
#pragma unroll
            for (int c = 0; c < C; ++c) p[o + c] = zv[c] + bt * p[o + c];
        }
    }
}

// x += alpha p ; r -= alpha q (q gathered from the operator's tile boxes) ;
// z0 = M^-1 r ; partial sums.
template <typename T, int C, int R, int NR>
__global__ __launch_bounds__(64 * R) void cg_update_kernel(Geo G, long long vpp, T *x, T *r, T *z,
                                                           const T *p, const T *q, const T *minv,
                                                           const ColState *cols, double *partial,
                                                           const int *prob_active) {
    constexpr int MS = (C == 3) ? 6 : 1;
    constexpr int REC = 2 + C * NR;
    constexpr int RF = (NR == 1) ? 3 : 0;
    const int prob = blockIdx.y;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double acc[REC];
#pragma unroll
    for (int k = 0; k < REC; ++k) acc[k] = 0.0;
    if (prob_active[prob] == 0) {
        wave_partials(acc, REC, partial, prob, R, w);
        return;
    }
    const T al = (T)cols[prob * R + w].alpha;
    const long long base = (long long)prob * vpp;
    const T *Mp = minv + (long long)prob * G.npts * MS;
    const T *qt = q + (long long)prob * ((long long)G.tiles_x * G.tiles_y * G.tiles_z) * (BOXPTS * R * C);
    const long long nblk = (G.npts + 63) / 64;
    for (long long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const long long pt = blk * 64 + lane;
        if (pt >= G.npts) continue;
        int X, Y, Z;
        lattice_xyz(G, pt, X, Y, Z);
        double qv[C];
        if (dirichlet_boundary(G, X, Y, Z)) {
#pragma unroll
            for (int c = 0; c < C; ++c) qv[c] = 0.0;
        } else {
            gather_tiles_col<T, C, R>(G, qt, X, Y, Z, w, qv);
        }
        T Mi[MS];
#pragma unroll
        for (int k = 0; k < MS; ++k) Mi[k] = Mp[pt * MS + k];
        double row[4] = {0, 0, 0, 0};
#pragma unroll
        for (int a = 0; a < NR; ++a) row[a] = G.rows[4 * pt + RF + a];
        const long long o = base + (pt * R + w) * C;
        T rv[C], zv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            x[o + c] += al * p[o + c];
            rv[c] = r[o + c] - al * (T)qv[c];
            r[o + c] = rv[c];
        }
        minv_apply<T, C>(Mi, rv, zv);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            z[o + c] = zv[c];
            acc[0] += (double)rv[c] * (double)zv[c];
            acc[1] += (double)rv[c] * (double)rv[c];
#pragma unroll
            for (int a = 0; a < NR; ++a) acc[2 + c * NR + a] += row[a] * (double)zv[c];
        }
    }
    wave_partials(acc, REC, partial, prob, R, w);
}

// Sum of partials[k][0..nparts) for k in [0, K) into sums[k]; 256 threads,
// wave q takes k = q, q + 4, ...; coalesced loads, 4 independent chains per lane.
__device__ inline void reduce_kmajor(const double *part, int K, int nparts, double *sums) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int k = wv; k < K; k += nw) {
        const double *src = part + (long long)k * nparts;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int i = lane;
        for (; i + 192 < nparts; i += 256) {
            s0 += src[i];
            s1 += src[i + 64];
            s2 += src[i + 128];
            s3 += src[i + 192];
        }
        for (; i < nparts; i += 64) s0 += src[i];
        const double s = wave_sum((s0 + s1) + (s2 + s3));
        if (lane == 0) sums[k] = s;
    }
}

// alpha = r.z / p.Kp per column (partials from the operator: [prob][R][tiles]).
template <int R>
__global__ void finish_alpha_kernel(const double *partial_pq, int nparts, ColState *cols) {
    const int prob = blockIdx.x;
    __shared__ double pq[R];
    reduce_kmajor(partial_pq + (long long)prob * R * nparts, R, nparts, pq);
    __syncthreads();
    if (threadIdx.x < R) {
        ColState &cs = cols[prob * R + threadIdx.x];
        const double v = pq[threadIdx.x];
        cs.pq = v;
        if (cs.done) {
            cs.alpha = 0.0;
        } else if (!(v > 0.0)) {
            cs.alpha = 0.0;
            cs.done = 2;
        } else {
            cs.alpha = cs.rz / v;
        }
    }
}

// rz = r.z0 - c^T (C M^-1 C^T)^-1 c, projection coefficients y, beta, convergence.
template <int C, int R>
__global__ void finish_beta_kernel(int nrow, const double *partial, int nparts, const double *ginv,
                                   double *ycoef, ColState *cols, int *prob_active, int first,
                                   double rtol2, int use_init, const ColState *mask) {
    const int prob = blockIdx.x;
    const int S = C * nrow;
    const int REC = 2 + S;
    __shared__ double sums[R * (2 + 3 * 4)];
    reduce_kmajor(partial + (long long)prob * R * REC * nparts, R * REC, nparts, sums);
    __syncthreads();
    const int lane = threadIdx.x;
    if (lane < R) {
        ColState &cs = cols[prob * R + lane];
        const double *c = &sums[lane * REC + 2];
        double rz = sums[lane * REC];
        if (S > 0) {
            const double *Gi = ginv + (long long)prob * S * S;
            double *yv = ycoef + ((long long)prob * R + lane) * S;
            double cy = 0.0;
            for (int I = 0; I < S; ++I) {
                double t = 0.0;
                for (int J = 0; J < S; ++J) t += Gi[I * S + J] * c[J];
                yv[I] = t;
                cy += c[I] * t;
            }
            rz -= cy;
        }
        if (rz < 0.0) rz = 0.0;
        const bool was_active = !cs.done;
        if (first) {
            cs.rz_init = rz;
            cs.beta = 0.0;
            cs.done = (mask != nullptr && mask[prob * R + lane].done) ? 1 : 0;
        } else {
            cs.beta = (cs.done || cs.rz == 0.0) ? 0.0 : rz / cs.rz;
            if (was_active) cs.iters += 1;
        }
        cs.rz_prev = cs.rz;
        cs.rz = rz;
        const double ref = use_init ? cs.rz_init : cs.eref;
        if (!cs.done && rz <= rtol2 * ref) cs.done = 1;
        if (cs.done) cs.beta = 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int act = 0;
        for (int rr = 0; rr < R; ++rr) act += cols[prob * R + rr].done ? 0 : 1;
        prob_active[prob] = act;
    }
}

// ------------------------------------------------------------------ launchers
#define CHOM_NR_DISPATCH(NRV, CALL)              \
    switch (NRV) {                               \
        case 0: { constexpr int NR = 0; CALL; } break; \
        case 1: { constexpr int NR = 1; CALL; } break; \
        default: { constexpr int NR = 4; CALL; } break; \
    }

template <typename T, int C, int R>
hipError_t launch_cg_init(const Geo &G, int nprob, long long vpp, const T *b, T *x, T *r, T *z,
                          const void *minv, double *partial, int nwg, hipStream_t s) {
    dim3 grid(nwg, nprob);
    const T *M = (const T *)minv;
    if (x == nullptr) {
        CHOM_NR_DISPATCH(G.nrow, (cg_init_kernel<T, C, R, NR, false><<<grid, 64 * R, 0, s>>>(G, vpp, b, x, r, z, M, partial)));
    } else {
        CHOM_NR_DISPATCH(G.nrow, (cg_init_kernel<T, C, R, NR, true><<<grid, 64 * R, 0, s>>>(G, vpp, b, x, r, z, M, partial)));
    }
    return hipGetLastError();
}

template <typename T, int C, int R>
hipError_t launch_cg_dir(const Geo &G, int nprob, long long vpp, T *r, const T *z, T *p, T *q,
                         const void *minv, const double *ycoef, const ColState *cols,
                         const int *prob_active, int nwg, hipStream_t s) {
    dim3 grid(nwg, nprob);
    const T *M = (const T *)minv;
    CHOM_NR_DISPATCH(G.nrow, (cg_dir_kernel<T, C, R, NR><<<grid, 64 * R, 0, s>>>(G, vpp, r, z, p, q, M, ycoef, cols, prob_active)));
    return hipGetLastError();
}

template <typename T, int C, int R>
hipError_t launch_cg_update(const Geo &G, int nprob, long long vpp, T *x, T *r, T *z, const T *p,
                            const T *q, const void *minv, const ColState *cols, double *partial,
                            const int *prob_active, int nwg, hipStream_t s) {
    dim3 grid(nwg, nprob);
    const T *M = (const T *)minv;
    CHOM_NR_DISPATCH(G.nrow, (cg_update_kernel<T, C, R, NR><<<grid, 64 * R, 0, s>>>(G, vpp, x, r, z, p, q, M, cols, partial, prob_active)));
    return hipGetLastError();
}

template <int C, int R>
hipError_t launch_finish_alpha(int nprob, const double *partial_pq, int nparts, ColState *cols,
                               hipStream_t s) {
    finish_alpha_kernel<R><<<nprob, 256, 0, s>>>(partial_pq, nparts, cols);
    return hipGetLastError();
}

template <int C, int R>
hipError_t launch_finish_beta(int nprob, int nrow, const double *partial, int nparts,
                              const double *ginv, double *ycoef, ColState *cols, int *prob_active,
                              int first, double rtol2, int use_init, hipStream_t s) {
    finish_beta_kernel<C, R><<<nprob, 256, 0, s>>>(nrow, partial, nparts, ginv, ycoef, cols,
                                                      prob_active, first, rtol2, use_init, nullptr);
    return hipGetLastError();
}

template <int C, int R>
hipError_t launch_finish_beta_masked(int nprob, int nrow, const double *partial, int nparts,
                                     const double *ginv, double *ycoef, ColState *cols,
                                     int *prob_active, double rtol2, const ColState *mask,
                                     hipStream_t s) {
    finish_beta_kernel<C, R><<<nprob, 256, 0, s>>>(nrow, partial, nparts, ginv, ycoef, cols,
                                                      prob_active, 1, rtol2, 1, mask);
    return hipGetLastError();
}


// Outer (refinement) residual projected as a vector: r64 <- r64 - C^T y with
// y = (C M^-1 C^T)^-1 C M^-1 r64 from the previous reduction, r32 = (float) r64,
// and the partial sums [r.z0, r.r, C z0] of the projected residual.  Taking the
// norm of the projected vector keeps the multiplier forces of the exact
// solution out of the FP64 stopping test.
template <int C, int R, int NR>
__global__ __launch_bounds__(64 * R) void proj_resid_kernel(Geo G, long long vpp, double *r64, float *r32,
                                                            const double *minv64, const double *ycoef,
                                                            double *partial) {
    constexpr int MS = (C == 3) ? 6 : 1;
    constexpr int REC = 2 + C * NR;
    constexpr int S = C * NR;
    constexpr int RF = (NR == 1) ? 3 : 0;
    const int prob = blockIdx.y;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double acc[REC];
#pragma unroll
    for (int k = 0; k < REC; ++k) acc[k] = 0.0;
    double yv[S > 0 ? S : 1];
#pragma unroll
    for (int k = 0; k < S; ++k) yv[k] = ycoef[((long long)prob * R + w) * S + k];
    const long long base = (long long)prob * vpp;
    const double *Mp = minv64 + (long long)prob * G.npts * MS;
    const long long nblk = (G.npts + 63) / 64;
    for (long long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const long long pt = blk * 64 + lane;
        if (pt >= G.npts) continue;
        double Mi[MS];
#pragma unroll
        for (int k = 0; k < MS; ++k) Mi[k] = Mp[pt * MS + k];
        double row[4] = {0, 0, 0, 0};
#pragma unroll
        for (int a = 0; a < NR; ++a) row[a] = G.rows[4 * pt + RF + a];
        const long long o = base + (pt * R + w) * C;
        double rv[C], zv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            double ct = 0.0;
#pragma unroll
            for (int a = 0; a < NR; ++a) ct += row[a] * yv[c * NR + a];
            rv[c] = r64[o + c] - ct;
            r64[o + c] = rv[c];
            r32[o + c] = (float)rv[c];
        }
        minv_apply<double, C>(Mi, rv, zv);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            acc[0] += rv[c] * zv[c];
            acc[1] += rv[c] * rv[c];
#pragma unroll
            for (int a = 0; a < NR; ++a) acc[2 + c * NR + a] += row[a] * zv[c];
        }
    }
    wave_partials(acc, REC, partial, prob, R, w);
}

template <int C, int R>
hipError_t launch_proj_resid(const Geo &G, int nprob, long long vpp, double *r64, float *r32,
                             const double *minv64, const double *ycoef, double *partial, int nwg,
                             hipStream_t s) {
    dim3 grid(nwg, nprob);
    CHOM_NR_DISPATCH(G.nrow, (proj_resid_kernel<C, R, NR><<<grid, 64 * R, 0, s>>>(G, vpp, r64, r32, minv64, ycoef, partial)));
    return hipGetLastError();
}

// ------------------------------------------------------------------ refinement helpers
template <int C, int R>
__global__ void residual64_kernel(Geo G, long long vpp, const double *b, const double *q64t, double *r64, float *r32) {
    constexpr int RC = R * C;
    const int prob = blockIdx.y;
    const double *qt = q64t ? q64t + (long long)prob * ((long long)G.tiles_x * G.tiles_y * G.tiles_z) * (BOXPTS * RC) : nullptr;
    long long p0, p1;
    {
        const long long per = (G.npts + gridDim.x - 1) / gridDim.x;
        p0 = blockIdx.x * per;
        p1 = p0 + per < G.npts ? p0 + per : G.npts;
    }
    for (long long pt = p0 + threadIdx.x; pt < p1; pt += blockDim.x) {
        int X, Y, Z;
        lattice_xyz(G, pt, X, Y, Z);
        double qv[RC];
        for (int v = 0; v < RC; ++v) qv[v] = 0.0;
        if (qt != nullptr && !dirichlet_boundary(G, X, Y, Z))
            for (int w = 0; w < R; ++w) gather_tiles_col<double, C, R>(G, qt, X, Y, Z, w, qv + w * C);
        const long long o = (long long)prob * vpp + pt * RC;
        for (int v = 0; v < RC; ++v) {
            const double val = b[o + v] - qv[v];
            r64[o + v] = val;
            if (r32) r32[o + v] = (float)val;
        }
    }
}

template <int C, int R>
__global__ void axpy_x64_kernel(long long total, double *x64, const float *d32) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x)
        x64[i] += (double)d32[i];
}

static inline int flat_grid(long long total) {
    long long g = (total + 255) / 256;
    return (int)(g < 16384 ? (g < 1 ? 1 : g) : 16384);
}

template <int C, int R>
hipError_t launch_residual64(const Geo &G, int nprob, long long vpp, const double *b,
                             const double *q64t, double *r64, float *r32, hipStream_t s) {
    const long long g = (G.npts + 511) / 512;
    dim3 grid((unsigned)(g < 1 ? 1 : (g > 1024 ? 1024 : g)), nprob);
    residual64_kernel<C, R><<<grid, 256, 0, s>>>(G, vpp, b, q64t, r64, r32);
    return hipGetLastError();
}

template <int C, int R>
hipError_t launch_axpy_x64(int nprob, long long vpp, double *x64, const float *d32, hipStream_t s) {
    const long long total = vpp * nprob;
    axpy_x64_kernel<C, R><<<flat_grid(total), 256, 0, s>>>(total, x64, d32);
    return hipGetLastError();
}

// Projection of the FP64 solution onto ker(C): x -= M^-1 C^T (C M^-1 C^T)^-1 C x.
template <int C, int R, int NR>
__global__ void cx_partial_kernel(Geo G, long long vpp, const double *x, double *partial) {
    constexpr int S = C * NR;
    constexpr int RF = (NR == 1) ? 3 : 0;
    const int prob = blockIdx.y;
    double acc[R * S];
#pragma unroll
    for (int k = 0; k < R * S; ++k) acc[k] = 0.0;
    long long p0, p1;
    point_range(G.npts, p0, p1);
    for (long long pt = p0 + threadIdx.x; pt < p1; pt += blockDim.x) {
        double row[4] = {0, 0, 0, 0};
#pragma unroll
        for (int a = 0; a < NR; ++a) row[a] = G.rows[4 * pt + RF + a];
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
            const long long o = (long long)prob * vpp + (pt * R + rr) * C;
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int a = 0; a < NR; ++a) acc[rr * S + c * NR + a] += row[a] * x[o + c];
        }
    }
    block_reduce_store<R * S>(acc, partial + ((long long)prob * gridDim.x + blockIdx.x) * R * S);
}

template <int C, int R, int NR>
__global__ void cx_finish_kernel(const double *partial, int nparts, const double *ginv, double *ycoef) {
    constexpr int S = C * NR;
    const int prob = blockIdx.x;
    const int lane = threadIdx.x;
    __shared__ double sums[R * S];
    for (int k = 0; k < R * S; ++k) {
        double s = 0.0;
        for (int w = lane; w < nparts; w += 64) s += partial[((long long)prob * nparts + w) * R * S + k];
        s = wave_sum(s);
        if (lane == 0) sums[k] = s;
    }
    __syncthreads();
    if (lane < R) {
        const double *Gi = ginv + (long long)prob * S * S;
        for (int I = 0; I < S; ++I) {
            double t = 0.0;
            for (int J = 0; J < S; ++J) t += Gi[I * S + J] * sums[lane * S + J];
            ycoef[((long long)prob * R + lane) * S + I] = t;
        }
    }
}

template <int C, int R, int NR>
__global__ void cx_correct_kernel(Geo G, long long vpp, double *x, const double *minv64, const double *ycoef) {
    constexpr int MS = (C == 3) ? 6 : 1;
    constexpr int S = C * NR;
    constexpr int RF = (NR == 1) ? 3 : 0;
    const int prob = blockIdx.y;
    long long p0, p1;
    point_range(G.npts, p0, p1);
    const double *yv = ycoef + (long long)prob * R * S;
    for (long long pt = p0 + threadIdx.x; pt < p1; pt += blockDim.x) {
        double Mi[MS];
        for (int k = 0; k < MS; ++k) Mi[k] = minv64[((long long)prob * G.npts + pt) * MS + k];
        double row[4] = {0, 0, 0, 0};
        for (int a = 0; a < NR; ++a) row[a] = G.rows[4 * pt + RF + a];
        for (int rr = 0; rr < R; ++rr) {
            double ct[C], corr[C];
            for (int c = 0; c < C; ++c) {
                ct[c] = 0.0;
                for (int a = 0; a < NR; ++a) ct[c] += row[a] * yv[rr * S + c * NR + a];
            }
            minv_apply<double, C>(Mi, ct, corr);
            const long long o = (long long)prob * vpp + (pt * R + rr) * C;
            for (int c = 0; c < C; ++c) x[o + c] -= corr[c];
        }
    }
}

template <int C, int R>
hipError_t launch_project(const Geo &G, int nprob, long long vpp, double *x64, const double *minv64,
                          const double *ginv64, double *partial, int nwg, hipStream_t s) {
    if (G.nrow == 0) return hipSuccess;
    dim3 grid(nwg, nprob);
    double *ycoef = partial + (long long)nprob * nwg * R * C * 4;
    if (G.nrow == 1) {
        cx_partial_kernel<C, R, 1><<<grid, VEC_BS, 0, s>>>(G, vpp, x64, partial);
        cx_finish_kernel<C, R, 1><<<nprob, FIN_BS, 0, s>>>(partial, nwg, ginv64, ycoef);
        cx_correct_kernel<C, R, 1><<<grid, VEC_BS, 0, s>>>(G, vpp, x64, minv64, ycoef);
    } else {
        cx_partial_kernel<C, R, 4><<<grid, VEC_BS, 0, s>>>(G, vpp, x64, partial);
        cx_finish_kernel<C, R, 4><<<nprob, FIN_BS, 0, s>>>(partial, nwg, ginv64, ycoef);
        cx_correct_kernel<C, R, 4><<<grid, VEC_BS, 0, s>>>(G, vpp, x64, minv64, ycoef);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ instantiations
#define CHOM_INST(T, C, R)                                                                                         \
    template hipError_t launch_cg_init<T, C, R>(const Geo &, int, long long, const T *, T *, T *, T *, const void *, \
                                                double *, int, hipStream_t);                                      \
    template hipError_t launch_cg_dir<T, C, R>(const Geo &, int, long long, T *, const T *, T *, T *, const void *, \
                                               const double *, const ColState *, const int *, int, hipStream_t);  \
    template hipError_t launch_cg_update<T, C, R>(const Geo &, int, long long, T *, T *, T *, const T *, const T *, \
                                                  const void *, const ColState *, double *, const int *, int,      \
                                                  hipStream_t);
CHOM_INST(double, 3, 6)
CHOM_INST(float, 3, 6)
CHOM_INST(double, 1, 3)
CHOM_INST(float, 1, 3)

#define CHOM_INST2(C, R)                                                                                          \
    template hipError_t launch_finish_alpha<C, R>(int, const double *, int, ColState *, hipStream_t);             \
    template hipError_t launch_finish_beta<C, R>(int, int, const double *, int, const double *, double *,         \
                                                 ColState *, int *, int, double, int, hipStream_t);               \
    template hipError_t launch_finish_beta_masked<C, R>(int, int, const double *, int, const double *, double *,  \
                                                        ColState *, int *, double, const ColState *, hipStream_t); \
    template hipError_t launch_residual64<C, R>(const Geo &, int, long long, const double *, const double *,      \
                                                double *, float *, hipStream_t);                                  \
    template hipError_t launch_axpy_x64<C, R>(int, long long, double *, const float *, hipStream_t);              \
    template hipError_t launch_proj_resid<C, R>(const Geo &, int, long long, double *, float *, const double *,   \
                                                const double *, double *, int, hipStream_t);                      \
    template hipError_t launch_project<C, R>(const Geo &, int, long long, double *, const double *,               \
                                             const double *, double *, int, hipStream_t);
CHOM_INST2(3, 6)
CHOM_INST2(1, 3)

}  // namespace chom
