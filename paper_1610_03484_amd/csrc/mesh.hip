// Plain-weave RVE generator and yarn tagger (GPU).
//
// Kuhn lattice of an n^3 grid on the unit cube; the yarns are the synthetic
// workload's four sinusoidal yarns with elliptical sections (the paper builds
// its RVE from elliptical yarn sections on spline paths, Sec. 1 and Table 1;
// it takes fibre directions from a potential-flow solve, Sec. 6, replaced here
// by the analytic centreline tangent).
#include "common.h"
#include "internal.h"

namespace chom {

__global__ void gen_vertices_kernel(int n, double *coords) {
    const long long nv = (long long)(n + 1) * (n + 1) * (n + 1);
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < nv;
         v += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(v % (n + 1));
        const int j = (int)((v / (n + 1)) % (n + 1));
        const int k = (int)(v / ((long long)(n + 1) * (n + 1)));
        coords[3 * v + 0] = (double)i / (double)n;
        coords[3 * v + 1] = (double)j / (double)n;
        coords[3 * v + 2] = (double)k / (double)n;
    }
}

// Ellipse test value of yarn y at centroid c (1 on the boundary).
__device__ inline double yarn_f(int y, const double c[3], double tang[3]) {
    const double two_pi = 6.283185307179586;
    const double phase = (y & 1) ? 3.141592653589793 : 0.0;
    const double off = (y & 1) ? 0.75 : 0.25;
    double s, co, d_in, zc;
    if (y < 2) {  // warp: along x, section in the y-z plane
        sincos(__dmul_rn(two_pi, c[0]) + phase, &s, &co);
        zc = __dadd_rn(0.5, __dmul_rn(0.12, s));
        d_in = (c[1] - off) / 0.2;
        tang[0] = 1.0;
        tang[1] = 0.0;
        tang[2] = __dmul_rn(0.12 * two_pi, co);
    } else {      // weft: along y, section in the x-z plane
        sincos(__dmul_rn(two_pi, c[1]) + phase, &s, &co);
        zc = __dsub_rn(0.5, __dmul_rn(0.12, s));
        d_in = (c[0] - off) / 0.2;
        tang[0] = 0.0;
        tang[1] = 1.0;
        tang[2] = -__dmul_rn(0.12 * two_pi, co);
    }
    const double d_z = (c[2] - zc) / 0.06;
    return __dadd_rn(__dmul_rn(d_in, d_in), __dmul_rn(d_z, d_z));
}

__global__ void gen_tets_kernel(int n, int32_t *tets, int8_t *phase, double *axis) {
    const long long nt = 6LL * n * n * n;
    const int n1 = n + 1;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nt;
         e += (long long)gridDim.x * blockDim.x) {
        const int t = (int)(e % 6);
        const long long cell = e / 6;
        const int ci = (int)(cell % n), cj = (int)((cell / n) % n), ck = (int)(cell / ((long long)n * n));
        int p0, p1;
        kuhn_perm(t, p0, p1);
        int v[4][3] = {{ci, cj, ck}, {ci, cj, ck}, {ci, cj, ck}, {ci + 1, cj + 1, ck + 1}};
        v[1][p0] += 1;
        v[2][p0] += 1;
        v[2][p1] += 1;
        double cen[3];
        double x[4][3];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            tets[4 * e + a] = v[a][0] + n1 * (v[a][1] + n1 * v[a][2]);
#pragma unroll
            for (int d = 0; d < 3; ++d) x[a][d] = (double)v[a][d] / (double)n;
        }
#pragma unroll
        for (int d = 0; d < 3; ++d)
            cen[d] = __dmul_rn(__dadd_rn(__dadd_rn(__dadd_rn(x[0][d], x[1][d]), x[2][d]), x[3][d]), 0.25);
        int ph = 0;
        double ax[3] = {0.0, 0.0, 0.0};
        for (int y = 0; y < 4 && ph == 0; ++y) {
            double tang[3];
            const double f = yarn_f(y, cen, tang);
            if (f <= 1.0) {
                ph = y + 1;
                const double nr = sqrt(tang[0] * tang[0] + tang[1] * tang[1] + tang[2] * tang[2]);
                ax[0] = tang[0] / nr;
                ax[1] = tang[1] / nr;
                ax[2] = tang[2] / nr;
            }
        }
        phase[e] = (int8_t)ph;
        axis[3 * e + 0] = ax[0];
        axis[3 * e + 1] = ax[1];
        axis[3 * e + 2] = ax[2];
    }
}

// Tags of any tet mesh of the unit cube: the same yarn test at the centroid
// (summed in vertex order, then scaled by 1/4) as the lattice generator.
__global__ void tag_tets_kernel(long long nt, const double *coords, const int32_t *tets, int8_t *phase, double *axis) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nt;
         e += (long long)gridDim.x * blockDim.x) {
        double cen[3];
        for (int d = 0; d < 3; ++d) {
            const double x0 = coords[3LL * tets[4 * e] + d], x1 = coords[3LL * tets[4 * e + 1] + d];
            const double x2 = coords[3LL * tets[4 * e + 2] + d], x3 = coords[3LL * tets[4 * e + 3] + d];
            cen[d] = __dmul_rn(__dadd_rn(__dadd_rn(__dadd_rn(x0, x1), x2), x3), 0.25);
        }
        int ph = 0;
        double ax[3] = {0.0, 0.0, 0.0};
        for (int y = 0; y < 4 && ph == 0; ++y) {
            double tang[3];
            const double f = yarn_f(y, cen, tang);
            if (f <= 1.0) {
                ph = y + 1;
                const double nr = sqrt(tang[0] * tang[0] + tang[1] * tang[1] + tang[2] * tang[2]);
                ax[0] = tang[0] / nr;
                ax[1] = tang[1] / nr;
                ax[2] = tang[2] / nr;
            }
        }
        phase[e] = (int8_t)ph;
        axis[3 * e + 0] = ax[0];
        axis[3 * e + 1] = ax[1];
        axis[3 * e + 2] = ax[2];
    }
}

hipError_t launch_tag(long long nt, const double *coords, const int32_t *tets, int8_t *phase, double *axis,
                      hipStream_t s) {
    const long long g = (nt + 255) / 256;
    tag_tets_kernel<<<(int)(g < 65535 ? (g < 1 ? 1 : g) : 65535), 256, 0, s>>>(nt, coords, tets, phase, axis);
    return hipGetLastError();
}

hipError_t launch_generate(int n, double *coords, int32_t *tets, int8_t *phase, double *axis,
                           hipStream_t s) {
    const long long nv = (long long)(n + 1) * (n + 1) * (n + 1);
    const long long nt = 6LL * n * n * n;
    const int bs = 256;
    const int gv = (int)((nv + bs - 1) / bs < 65535 ? (nv + bs - 1) / bs : 65535);
    const int gt = (int)((nt + bs - 1) / bs < 65535 ? (nt + bs - 1) / bs : 65535);
    gen_vertices_kernel<<<gv, bs, 0, s>>>(n, coords);
    gen_tets_kernel<<<gt, bs, 0, s>>>(n, tets, phase, axis);
    return hipGetLastError();
}

}  // namespace chom
