// Per-RVE and per-problem setup kernels: element data, constraint rows,
// block-Jacobi preconditioner, Gram matrices of the constraint projection and
// the load vectors of the unit macro strains / gradients.
#include "common.h"
#include "internal.h"

namespace chom {

static inline int grid_for(long long work, int bs, int cap = 16384) {
    long long g = (work + bs - 1) / bs;
    if (g < 1) g = 1;
    return (int)(g < cap ? g : cap);
}

// ------------------------------------------------------------------ element data
__global__ void element_setup_kernel(Geo G, const double *coords, const int8_t *phase,
                                     const double *axis, double4 *elem64, float4 *elem32,
                                     double *geo64, float *geo32, int *bad) {
    const int n = G.n, n1 = n + 1;
    const long long nt = 6LL * n * n * n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nt;
         e += (long long)gridDim.x * blockDim.x) {
        const int ph = phase[e];
        double a[3] = {axis[3 * e], axis[3 * e + 1], axis[3 * e + 2]};
        if (ph == 0) a[0] = a[1] = a[2] = 0.0;
        elem64[e] = make_double4(a[0], a[1], a[2], (double)ph);
        elem32[e] = make_float4((float)a[0], (float)a[1], (float)a[2], (float)ph);
        if (geo64 == nullptr) continue;
        const int t = (int)(e % 6);
        const long long cell = e / 6;
        const int ci = (int)(cell % n), cj = (int)((cell / n) % n), ck = (int)(cell / ((long long)n * n));
        int p0, p1;
        kuhn_perm(t, p0, p1);
        int v[4][3] = {{ci, cj, ck}, {ci, cj, ck}, {ci, cj, ck}, {ci + 1, cj + 1, ck + 1}};
        v[1][p0] += 1;
        v[2][p0] += 1;
        v[2][p1] += 1;
        double x[4][3];
        for (int k = 0; k < 4; ++k) {
            const long long id = v[k][0] + (long long)n1 * (v[k][1] + (long long)n1 * v[k][2]);
            for (int d = 0; d < 3; ++d) x[k][d] = coords[3 * id + d];
        }
        double J[3][3];  // columns x1-x0, x2-x0, x3-x0
        for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) J[d][c] = x[c + 1][d] - x[0][d];
        const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        // expected orientation: sign of the axis permutation (even: t = 0, 3, 4)
        const double sgn = (t == 0 || t == 3 || t == 4) ? 1.0 : -1.0;
        if (!(det * sgn > 0.0)) atomicAdd(bad, 1);
        const double id = 1.0 / det;
        // rows of J^-1 are the gradients of lam_1..3
        double Ji[3][3];
        Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
        Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
        Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
        double *g64 = geo64 + e * 10;
        float *g32 = geo32 + e * 10;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                g64[3 * i + j] = Ji[i][j];
                g32[3 * i + j] = (float)Ji[i][j];
            }
        g64[9] = fabs(det) / 6.0;
        g32[9] = (float)(fabs(det) / 6.0);
    }
}

hipError_t launch_element_setup(const Geo &G, const double *coords, const int32_t *,
                                const int8_t *phase, const double *axis, double4 *elem64,
                                float4 *elem32, double *geo64, float *geo32, int *bad_count,
                                hipStream_t s) {
    const long long nt = 6LL * G.n * G.n * G.n;
    element_setup_kernel<<<grid_for(nt, 256), 256, 0, s>>>(G, coords, phase, axis, elem64, elem32,
                                                           geo64, geo32, bad_count);
    return hipGetLastError();
}

// Tet handled by thread index u of a scatter kernel: threads run type-major
// (u = t * cells + cell), so the 64 tets of a wave are of one type in 64
// neighbouring cells and their atomic adds mostly hit different points.
__device__ inline long long scatter_tet(long long u, long long ncells) {
    const long long t = u / ncells;
    return (u - t * ncells) * 6 + t;
}

// Decode tet id -> (cell coords, type) and the 10 DOF lattice points.
__device__ inline void tet_points(const Geo &G, long long e, int &t, int P[10][3]) {
    const int n = G.n;
    t = (int)(e % 6);
    const long long cell = e / 6;
    const int ci = (int)(cell % n), cj = (int)((cell / n) % n), ck = (int)(cell / ((long long)n * n));
    int off[10][3];
    p2_dof_offsets(t, off);
    for (int k = 0; k < 10; ++k) {
        P[k][0] = 2 * ci + off[k][0];
        P[k][1] = 2 * cj + off[k][1];
        P[k][2] = 2 * ck + off[k][2];
    }
}

// ------------------------------------------------------------------ constraint rows
// Per DOF: int grad(phi) dV (3) and int phi dV (1).  For interior DOFs the
// gradient integral vanishes; for boundary DOFs it is the surface moment
// int phi n dS of the uniform-traction rows (divergence theorem).
__global__ void rows_kernel(Geo G, double *rows) {
    const long long nt = 6LL * G.n * G.n * G.n;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nt;
         e += (long long)gridDim.x * blockDim.x) {
        int t, P[10][3];
        tet_points(G, e, t, P);
        double g[4][3], vol;
        GeoSel<double>::get(G, e, t, g, vol);
        for (int k = 0; k < 10; ++k) {
            double m[3], w;
            if (k < 4) {
                for (int d = 0; d < 3; ++d) m[d] = vol * g[k][d];
                w = 0.25 * vol;
            } else {
                int a, b;
                edge_verts(k - 4, a, b);
                for (int d = 0; d < 3; ++d) m[d] = vol * (g[a][d] + g[b][d]);
                w = 0.2 * vol;
            }
            const long long idx = lat_index(G, P[k][0], P[k][1], P[k][2]);
            for (int d = 0; d < 3; ++d) atomicAdd(&rows[4 * idx + d], m[d]);
            atomicAdd(&rows[4 * idx + 3], w);
        }
    }
}

hipError_t launch_rows(const Geo &G, double *rows, hipStream_t s) {
    hipError_t err = hipMemsetAsync(rows, 0, sizeof(double) * 4 * G.npts, s);
    if (err != hipSuccess) return err;
    if (G.p != 2) return launch_rows_hp(G, rows, s);
    const long long nt = 6LL * G.n * G.n * G.n;
    rows_kernel<<<grid_for(nt, 256), 256, 0, s>>>(G, rows);
    return hipGetLastError();
}

// ------------------------------------------------------------------ preconditioner
// Point-block Jacobi: the blocks of diag(K) come, for order 2, from the
// operator kernel's diagonal mode (tile boxes, LDS accumulation) summed per
// point here; Dirichlet points get a zero block (and a zero inverse).
template <int C>
__global__ void diag_gather_kernel(const Geo *geos, const Prob *probs, const double *q, double *diag) {
    constexpr int MS = (C == 3) ? 6 : 1;
    constexpr int R = (C == 3) ? 6 : 3;
    constexpr int RG = (C == 3) ? 2 : 1;
    const Prob &P = probs[blockIdx.y];
    const Geo &G = geos[P.geo];
    double *D = diag + P.doff * MS;
    const double *qt = q + P.qoff;
    for (long long pt = blockIdx.x * (long long)blockDim.x + threadIdx.x; pt < G.npts;
         pt += (long long)gridDim.x * blockDim.x) {
        int X, Y, Z;
        lattice_xyz(G, pt, X, Y, Z);
        double out[MS];
#pragma unroll
        for (int v = 0; v < MS; ++v) out[v] = 0.0;
        if (!dirichlet_boundary(G, X, Y, Z)) {
            if constexpr (C == 3) {
                gather_tiles_col<double, 3, R>(G, qt, RG, X, Y, Z, 0, out);
                gather_tiles_col<double, 3, R>(G, qt, RG, X, Y, Z, 1, out + 3);
            } else {
                gather_tiles_col<double, 1, R>(G, qt, RG, X, Y, Z, 0, out);
            }
        }
#pragma unroll
        for (int v = 0; v < MS; ++v) D[pt * MS + v] = out[v];
    }
}

template <int C>
__global__ void invert_diag_kernel(long long total, const double *diag, double *minv64, float *minv32) {
    constexpr int MS = (C == 3) ? 6 : 1;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const double *d = diag + i * MS;
        double *o = minv64 + i * MS;
        float *o32 = minv32 + i * MS;
        if constexpr (C == 3) {
            const double a = d[0], b = d[1], c = d[2], xy = d[3], yz = d[4], xz = d[5];
            const double c00 = b * c - yz * yz, c11 = a * c - xz * xz, c22 = a * b - xy * xy;
            const double c01 = xz * yz - xy * c, c12 = xy * xz - a * yz, c02 = xy * yz - b * xz;
            const double det = a * c00 + xy * c01 + xz * c02;
            double r[6] = {0, 0, 0, 0, 0, 0};
            if (det > 0.0) {
                const double id = 1.0 / det;
                r[0] = c00 * id; r[1] = c11 * id; r[2] = c22 * id;
                r[3] = c01 * id; r[4] = c12 * id; r[5] = c02 * id;
            }
            for (int k = 0; k < 6; ++k) {
                o[k] = r[k];
                o32[k] = (float)r[k];
            }
        } else {
            const double r = d[0] > 0.0 ? 1.0 / d[0] : 0.0;
            o[0] = r;
            o32[0] = (float)r;
        }
    }
}

template <int C>
hipError_t launch_precond(const Launch &L, long long total_pts, double *diag, double *minv64, float *minv32,
                          double *qscratch, hipStream_t s) {
    constexpr int MS = (C == 3) ? 6 : 1;
    constexpr int R = (C == 3) ? 6 : 3;
    hipError_t err;
    if (L.order != 2) {
        err = hipMemsetAsync(diag, 0, sizeof(double) * MS * total_pts, s);
        if (err != hipSuccess) return err;
        err = launch_diag_hp<C>(L, diag, s);
        if (err != hipSuccess) return err;
    } else {
        err = launch_diag_operator<C, R>(L, qscratch, s);
        if (err != hipSuccess) return err;
        diag_gather_kernel<C><<<dim3(grid_for(L.max_tets / 6 + 1, 256, 1024), L.nprob), 256, 0, s>>>(L.geos, L.probs,
                                                                                                    qscratch, diag);
    }
    invert_diag_kernel<C><<<grid_for(total_pts, 256), 256, 0, s>>>(total_pts, diag, minv64, minv32);
    return hipGetLastError();
}
template hipError_t launch_precond<3>(const Launch &, long long, double *, double *, float *, double *, hipStream_t);
template hipError_t launch_precond<1>(const Launch &, long long, double *, double *, float *, double *, hipStream_t);

// ------------------------------------------------------------------ Gram matrices
// G[(i,a),(j,b)] = sum_pt row_a(pt) row_b(pt) Minv_pt[i][j] for the rows of the
// boundary condition (periodic: int phi; Neumann: int grad(phi), int phi), with
// the FP64 and with the FP32 preconditioner.  Unique sums: sym(Minv) x sym(rows).
constexpr int GRAM_CHUNK = 256;

template <int C>
__global__ void gram_partial_kernel(const Geo *geos, const Prob *probs, const double *minv64, const float *minv32,
                                    double *partial) {
    constexpr int MS = (C == 3) ? 6 : 1;
    constexpr int NUMAX = 60;
    const Prob &P = probs[blockIdx.y];
    const Geo &G = geos[P.geo];
    const int nrow = G.nrow;
    const int rfirst = (nrow == 1) ? 3 : 0;  // periodic uses only int phi
    const int nRs = nrow * (nrow + 1) / 2;
    const int nU = MS * nRs;
    __shared__ double sm64[GRAM_CHUNK][MS];
    __shared__ double sm32[GRAM_CHUNK][MS];
    __shared__ double sr[GRAM_CHUNK][4];
    const int prob = blockIdx.y;
    const double *M64 = minv64 + P.doff * MS;
    const float *M32 = minv32 + P.doff * MS;
    // each thread owns unique sum u (two precisions)
    const int u = threadIdx.x;
    int mi = 0, ra = 0, rb = 0;
    if (u < nU) {
        mi = u / nRs;
        int rr = u % nRs;
        for (ra = 0; ra < nrow; ++ra) {
            if (rr < nrow - ra) { rb = ra + rr; break; }
            rr -= nrow - ra;
        }
    }
    double acc64 = 0.0, acc32 = 0.0;
    const long long per = (G.npts + gridDim.x - 1) / gridDim.x;
    const long long p0 = blockIdx.x * per;
    const long long p1 = (p0 + per < G.npts) ? p0 + per : G.npts;
    for (long long base = p0; base < p1; base += GRAM_CHUNK) {
        __syncthreads();
        const long long pt = base + threadIdx.x;
        if (threadIdx.x < GRAM_CHUNK) {
            if (pt < p1) {
                for (int k = 0; k < MS; ++k) {
                    sm64[threadIdx.x][k] = M64[pt * MS + k];
                    sm32[threadIdx.x][k] = (double)M32[pt * MS + k];
                }
                for (int k = 0; k < 4; ++k) sr[threadIdx.x][k] = G.rows[4 * pt + k];
            } else {
                for (int k = 0; k < MS; ++k) sm64[threadIdx.x][k] = sm32[threadIdx.x][k] = 0.0;
                for (int k = 0; k < 4; ++k) sr[threadIdx.x][k] = 0.0;
            }
        }
        __syncthreads();
        if (u < nU) {
            for (int q = 0; q < GRAM_CHUNK; ++q) {
                const double rp = sr[q][rfirst + ra] * sr[q][rfirst + rb];
                acc64 += rp * sm64[q][mi];
                acc32 += rp * sm32[q][mi];
            }
        }
    }
    if (u < nU) {
        double *out = partial + ((long long)prob * gridDim.x + blockIdx.x) * 2 * NUMAX;
        out[u] = acc64;
        out[NUMAX + u] = acc32;
    }
}

// Expand the unique sums of one problem, invert (Gauss-Jordan, pivoted), store.
// One workgroup per problem: the threads sum the partials of the S x S entries
// into LDS, one thread inverts.
template <int C>
__global__ __launch_bounds__(256) void gram_finish_kernel(const Geo *geos, const Prob *probs, int nprob, int nwg,
                                                          const double *partial, double *ginv64, double *ginv32,
                                                          int *bad, double *gmat) {
    constexpr int MS = (C == 3) ? 6 : 1;
    constexpr int NUMAX = 60;
    constexpr int SMAX = C * 4;
    __shared__ double A[12][24];
    __shared__ int ok_s, piv_s[2];
    const int prob = blockIdx.x;
    const int nrow = geos[probs[prob].geo].nrow;
    if (nrow == 0) return;
    const int nRs = nrow * (nrow + 1) / 2;
    const int S = C * nrow;
    for (int which = 0; which < 2; ++which) {
        for (int t = threadIdx.x; t < S * S; t += blockDim.x) {
            const int I = t / S, J = t % S;
            const int i = I / nrow, a = I % nrow, j = J / nrow, b = J % nrow;
            int mi;
            if (C == 3) {
                const int lo = i < j ? i : j, hi = i < j ? j : i;
                mi = (lo == hi) ? lo : (lo == 0 && hi == 1 ? 3 : (lo == 1 && hi == 2 ? 4 : 5));
            } else {
                mi = 0;
            }
            const int ra = a < b ? a : b, rb = a < b ? b : a;
            int ri = 0;
            for (int q = 0; q < ra; ++q) ri += nrow - q;
            ri += rb - ra;
            const int u = mi * nRs + ri;
            double sum = 0.0;
            for (int w = 0; w < nwg; ++w) sum += partial[((long long)prob * nwg + w) * 2 * NUMAX + which * NUMAX + u];
            A[I][J] = sum;
            A[I][S + J] = (I == J) ? 1.0 : 0.0;
            if (gmat != nullptr) gmat[((long long)which * nprob + prob) * SMAX * SMAX + I * S + J] = sum;
        }
        __syncthreads();
        const int ok = gauss_jordan_wg(A, S, piv_s);
        if (threadIdx.x == 0) {
            ok_s = ok;
            if (!ok) atomicAdd(bad, 1);
        }
        __syncthreads();
        double *out = (which == 0 ? ginv64 : ginv32) + (long long)prob * SMAX * SMAX;
        for (int t = threadIdx.x; t < S * S; t += blockDim.x) out[t] = ok_s ? A[t / S][S + t % S] : 0.0;
        __syncthreads();
    }
    (void)MS;
}

template <int C>
hipError_t launch_gram(const Launch &L, const double *minv64, const float *minv32, double *gram_partial, int nwg,
                       double *ginv64, double *ginv32, int *bad, hipStream_t s, double *gmat) {
    if (L.nr == 0) return hipSuccess;
    dim3 grid(nwg, L.nprob);
    gram_partial_kernel<C><<<grid, GRAM_CHUNK, 0, s>>>(L.geos, L.probs, minv64, minv32, gram_partial);
    gram_finish_kernel<C><<<L.nprob, 256, 0, s>>>(L.geos, L.probs, L.nprob, nwg, gram_partial, ginv64, ginv32, bad,
                                                  gmat);
    return hipGetLastError();
}
template hipError_t launch_gram<3>(const Launch &, const double *, const float *, double *, int, double *, double *, int *, hipStream_t, double *);
template hipError_t launch_gram<1>(const Launch &, const double *, const float *, double *, int, double *, double *, int *, hipStream_t, double *);

// ------------------------------------------------------------------ load vectors
// b_i = - int grad(phi_i) : C eps_k dV for the unit strains (or - int grad(phi_i) . k e_k
// for unit gradients), i.e. minus the stiffness times the interpolated linear
// field; also the energy of the linear field eps_k : C_e eps_k |e| (reference
// scale of the stopping test).
// Linear-field energies of the unit load cases from the striped accumulators
// (cleared afterwards).
template <int R>
__global__ void eref_kernel(double *acc_pq, ColState *cols) {
    const int prob = blockIdx.x;
    if (threadIdx.x < R) {
        double *a = acc_pq + ((long long)prob * R + threadIdx.x) * ACC_STRIPES;
        double v = 0.0;
        for (int st = 0; st < ACC_STRIPES; ++st) {
            v += a[st];
            a[st] = 0.0;
        }
        cols[prob * R + threadIdx.x].eref = v;
    }
}

// Order 2: the operator kernel in its load-vector mode writes the tile boxes of
// K x_lin (no global atomics) and b = -K x_lin is gathered from them; orders 3,
// 4 scatter per tet.
template <int C, int R>
hipError_t launch_rhs(const Launch &L, long long total_vals, double *b, ColState *cols, double *q64t,
                      double *acc_pq, hipStream_t s) {
    if (L.order != 2) {
        hipError_t err = hipMemsetAsync(b, 0, sizeof(double) * total_vals, s);
        if (err != hipSuccess) return err;
        return launch_rhs_hp<C, R>(L, b, cols, s);
    }
    hipError_t err = launch_zero(acc_pq, (long long)L.nprob * R * ACC_STRIPES, s);
    if (err != hipSuccess) return err;
    if ((err = launch_rhs_operator<C, R>(L, L.rg, q64t, acc_pq, s)) != hipSuccess) return err;
    if ((err = launch_residual64<C, R>(L, nullptr, q64t, b, nullptr, s)) != hipSuccess) return err;
    eref_kernel<R><<<L.nprob, 64, 0, s>>>(acc_pq, cols);
    return hipGetLastError();
}
template hipError_t launch_rhs<3, 6>(const Launch &, long long, double *, ColState *, double *, double *, hipStream_t);
template hipError_t launch_rhs<1, 3>(const Launch &, long long, double *, ColState *, double *, double *, hipStream_t);

}  // namespace chom
