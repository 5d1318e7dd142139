// Homogenisation average (paper Sec. 2, Eq. macro_stress and Eq. Eq_C_stress;
// Eq. eq_homo_flux for the scalar fields): for load case k,
//   sigma_bar_k = (1/V) sum_e C_e (eps_k |e| + int_e sym grad(u~_k) dV),
// accumulated in FP64 from the FP64 fluctuation.  Column k of C_bar is
// sigma_bar_k; K_bar and D_bar likewise with fluxes k_e (e_k |e| + int grad psi~).
// For the exact discrete fluctuation this equals the energy form
// (1/V) (x_i + u_i)^T K (x_k + u_k) (the residual of load case k vanishes on
// admissible u_i); for an iterate u = u* + e the plain average is off by a term
// linear in e, the energy form only by e_i^T K e_k.  The library therefore
// subtracts (1/V) u_i . r_k, r_k = b_k - K u_k the final projected residual.
#include "common.h"
#include "internal.h"

namespace chom {

template <int C, int R>
__global__ __launch_bounds__(256) void average_kernel(const Geo *geos, const Prob *probs, const double *x, double *partial) {
    constexpr int NC = (C == 3) ? 6 : 3;
    const int prob = blockIdx.y;
    const Prob &P = probs[prob];
    const Geo &G = geos[P.geo];
    const double *xp = x + P.voff;
    const long long nt = 6LL * G.n * G.n * G.n;
    double acc[R * NC];   // indexed with compile-time indices only (all loops over it unrolled)
#pragma unroll
    for (int k = 0; k < R * NC; ++k) acc[k] = 0.0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nt;
         e += (long long)gridDim.x * blockDim.x) {
        const int n = G.n;
        const int t = (int)(e % 6);
        const long long cell = e / 6;
        const int ci = (int)(cell % n), cj = (int)((cell / n) % n), ck = (int)(cell / ((long long)n * n));
        int off[10][3];
        p2_dof_offsets(t, off);
        double g[4][3], vol, a[3];
        int ph;
        GeoSel<double>::get(G, e, t, g, vol);
        GeoSel<double>::elem(G, e, a, ph);
        const double *m = P.mat64[ph ? 1 : 0];
        long long idx[10];
        double w[10][3];
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            idx[k] = lat_index(G, 2 * ci + off[k][0], 2 * cj + off[k][1], 2 * ck + off[k][2]);
            if (k < 4) {
                for (int d = 0; d < 3; ++d) w[k][d] = vol * g[k][d];
            } else {
                int a2, b2;
                edge_verts(k - 4, a2, b2);
                for (int d = 0; d < 3; ++d) w[k][d] = vol * (g[a2][d] + g[b2][d]);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double H[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};   // int grad(u~) dV
#pragma unroll
            for (int k = 0; k < 10; ++k)
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const double u = xp[(r * G.npts + idx[k]) * C + c];
                    for (int d = 0; d < 3; ++d) H[c][d] += u * w[k][d];
                }
            if constexpr (C == 3) {
                double eps[6] = {H[0][0], H[1][1], H[2][2], 0.5 * (H[0][1] + H[1][0]),
                                 0.5 * (H[1][2] + H[2][1]), 0.5 * (H[2][0] + H[0][2])};
                if (r < 3) eps[r] += vol; else eps[r] += 0.5 * vol;
                double s[6];
                stress_ti<double>(eps, a, m, s);
#pragma unroll
                for (int k = 0; k < 6; ++k) acc[r * NC + k] += s[k];
            } else {
                double gr[3] = {H[0][0], H[0][1], H[0][2]};
                gr[r] += vol;
                double q[3];
                flux_ti<double>(gr, a, m, q);
#pragma unroll
                for (int k = 0; k < 3; ++k) acc[r * NC + k] += q[k];
            }
        }
    }
    __shared__ double red[R * NC][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
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

// Residual correction of the average: u_l . r_k summed over the lattice for every
// pair of load cases (l, k), u the fluctuation and r = b - K u its projected
// residual.  Wave w takes u_w; partial[((prob * nwg + block) * R + l) * R + k].
template <int C, int R>
__global__ __launch_bounds__(64 * R) void residual_pair_kernel(const Geo *geos, const Prob *probs, const double *x,
                                                               const double *r, double *partial) {
    const int prob = blockIdx.y;
    const Prob &P = probs[prob];
    const Geo &G = geos[P.geo];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double acc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = 0.0;
    const double *xp = x + P.voff, *rp = r + P.voff;
    for (long long pt = blockIdx.x * 64LL + lane; pt < G.npts; pt += gridDim.x * 64LL) {
        double u[C];
#pragma unroll
        for (int c = 0; c < C; ++c) u[c] = xp[(w * G.npts + pt) * C + c];
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
            for (int c = 0; c < C; ++c) acc[k] += u[c] * rp[(k * G.npts + pt) * C + c];
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) partial[(((long long)prob * gridDim.x + blockIdx.x) * R + w) * R + k] = v;
    }
}

// out[prob][i][j] = (1/V) sum of partials: row i = stress/flux component, column j = load case.
// With `rpart` (residual_pair_kernel sums, nwg2 blocks) the entry becomes the
// energy form (1/V) (x_i + u_i)^T K (x_j + u_j) = sigma_bar_j[i] - (1/V) u_i . r_j
// (unit load cases in the stress/flux component order, so NC = R), and `corr`
// (nullable) receives (1/V) u_i . r_j: the gap between the plain average and the
// energy form, i.e. the Hill-Mandel defect of the computed fluctuation (zero for
// the exact discrete solution, Sec. 2).
template <int C, int R>
__global__ void average_finish_kernel(const Geo *geos, const Prob *probs, int nwg, const double *partial, int nwg2,
                                      const double *rpart, double *out, double *corr) {
    constexpr int NC = (C == 3) ? 6 : 3;
    static_assert(NC == R, "load cases are the unit strains / gradients");
    const int prob = blockIdx.x;
    const double volume = geos[probs[prob].geo].volume;
    const int lane = threadIdx.x;
    for (int k = 0; k < R * NC; ++k) {
        const int r = k / NC, i = k % NC;   // load case r, component i
        double s = 0.0, g = 0.0;
        for (int w = lane; w < nwg; w += 64) s += partial[((long long)prob * nwg + w) * R * NC + k];
        if (rpart != nullptr)
            for (int w = lane; w < nwg2; w += 64) g += rpart[(((long long)prob * nwg2 + w) * R + i) * R + r];
        s = wave_sum(s);
        g = wave_sum(g);
        if (lane == 0) {
            out[(long long)prob * NC * R + i * R + r] = (s - g) / volume;
            if (corr != nullptr) corr[(long long)prob * NC * R + i * R + r] = g / volume;
        }
    }
}

template <int C, int R>
hipError_t launch_average(const Launch &L, const double *x64, const double *r64, double *partial, int nwg,
                          double *out, hipStream_t s, double *corr) {
    dim3 grid(nwg, L.nprob);
    if (L.order != 2) {
        const hipError_t e = launch_average_partial_hp<C, R>(L, x64, partial, nwg, s);
        if (e != hipSuccess) return e;
    } else {
        average_kernel<C, R><<<grid, 256, 0, s>>>(L.geos, L.probs, x64, partial);
    }
    constexpr int NC = (C == 3) ? 6 : 3;
    double *rpart = r64 ? partial + (size_t)L.nprob * nwg * R * NC : nullptr;
    if (r64) residual_pair_kernel<C, R><<<grid, 64 * R, 0, s>>>(L.geos, L.probs, x64, r64, rpart);
    average_finish_kernel<C, R><<<L.nprob, FIN_BS, 0, s>>>(L.geos, L.probs, nwg, partial, nwg, rpart, out,
                                                           rpart ? corr : nullptr);
    return hipGetLastError();
}
template hipError_t launch_average<3, 6>(const Launch &, const double *, const double *, double *, int, double *,
                                        hipStream_t, double *);
template hipError_t launch_average<1, 3>(const Launch &, const double *, const double *, double *, int, double *,
                                        hipStream_t, double *);

}  // namespace chom
