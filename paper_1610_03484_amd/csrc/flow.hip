// Yarn directions from a potential-flow solve on each yarn (paper Sec. 6): the
// fibre direction of a yarn tet is the normalised gradient of a potential phi
// solving Laplace's equation on that yarn's tetrahedra alone, with phi = 0 on
// the yarn's vertices on the inlet face lo[d] of the cell, phi = 1 on those on
// the outlet face hi[d] (d the axis the yarn runs along) and no flux through
// the rest of its surface.  Linear (P1) elements on the Kuhn lattice: the
// stiffness couples a vertex only to its 14 Kuhn neighbours, so each yarn's
// system is a 15-point stencil on the vertex lattice (entry |e| g_a . g_b summed
// over the yarn's tets at the vertex, g the barycentric gradients from the
// vertex coordinates, so distorted lattices work too).
//
// Kernels: stencil assembly (one thread per vertex and yarn, gathering over the
// 24 tets at the vertex: no atomics); Jacobi-preconditioned CG in FP64 with one
// workgroup per yarn (a yarn holds a small fraction of the lattice; the
// iteration is latency-bound, so block barriers replace kernel launches); the
// per-tet gradient.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace chom {
namespace {

constexpr int FLOW_BS = 1024;
enum { V_OFF = 0, V_FREE = 1, V_INLET = 2, V_OUTLET = 3 };

struct FlowArgs {
    int n;                     // cells per side
    long long nv;              // (n + 1)^3 vertices
    const double *coords;      // [nv][3]
    const int8_t *phase;       // [6 n^3]
    const int *axis;           // [nyarn] coordinate the yarn runs along
    double *A;                 // [nyarn][nv][15] stencils
    int *flag;                 // [nyarn][nv]
    double *phi, *r, *p, *q;   // [nyarn][nv]
    int *iters;                // [nyarn] CG steps taken (negative: not converged)
};

__device__ inline int kuhn_slot(int dx, int dy, int dz) {
    for (int k = 0; k < MG_SLOTS; ++k) {
        int a, b, c;
        kuhn_offset(k, a, b, c);
        if (a == dx && b == dy && c == dz) return k;
    }
    return -1;
}

// Vertex (lattice) indices of tet `type` of the cell at (ci, cj, ck).
__device__ inline void tet_lattice(int ci, int cj, int ck, int type, int v[4][3]) {
    int p0, p1;
    kuhn_perm(type, p0, p1);
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

__device__ inline long long vid(int i, int j, int k, int n) {
    return i + (long long)(n + 1) * (j + (long long)(n + 1) * k);
}

// Barycentric gradients and volume of a tet from its vertex coordinates.
__device__ inline double tet_grads(const double *coords, const long long id[4], double g[4][3]) {
    double x[4][3];
    for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d) x[a][d] = coords[3 * id[a] + d];
    double J[3][3];   // columns: edges from vertex 0
    for (int d = 0; d < 3; ++d)
        for (int e = 0; e < 3; ++e) J[d][e] = x[e + 1][d] - x[0][d];
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    const double id_ = 1.0 / det;
    // rows of J^-1 (the adjugate over det) are the gradients of lambda_1..3
    g[1][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id_;
    g[1][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id_;
    g[1][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id_;
    g[2][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id_;
    g[2][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id_;
    g[2][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id_;
    g[3][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id_;
    g[3][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id_;
    g[3][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id_;
    for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
    return fabs(det) / 6.0;
}

// Stencil row of vertex v for yarn blockIdx.y: sum over the yarn's tets at v.
__global__ __launch_bounds__(256) void flow_assemble_kernel(FlowArgs F) {
    const int y = blockIdx.y, n = F.n;
    const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (v >= F.nv) return;
    const int i = (int)(v % (n + 1)), j = (int)((v / (n + 1)) % (n + 1)), k = (int)(v / ((long long)(n + 1) * (n + 1)));
    double row[MG_SLOTS];
    for (int s = 0; s < MG_SLOTS; ++s) row[s] = 0.0;
    bool touched = false;
    for (int dk = -1; dk <= 0; ++dk)
        for (int dj = -1; dj <= 0; ++dj)
            for (int di = -1; di <= 0; ++di) {
                const int ci = i + di, cj = j + dj, ck = k + dk;
                if (ci < 0 || cj < 0 || ck < 0 || ci >= n || cj >= n || ck >= n) continue;
                const long long cell = ci + (long long)n * (cj + (long long)n * ck);
                for (int t = 0; t < 6; ++t) {
                    if (F.phase[cell * 6 + t] != y + 1) continue;
                    int lv[4][3];
                    tet_lattice(ci, cj, ck, t, lv);
                    int a = -1;
                    for (int b = 0; b < 4; ++b)
                        if (lv[b][0] == i && lv[b][1] == j && lv[b][2] == k) a = b;
                    if (a < 0) continue;
                    long long id[4];
                    for (int b = 0; b < 4; ++b) id[b] = vid(lv[b][0], lv[b][1], lv[b][2], n);
                    double g[4][3];
                    const double vol = tet_grads(F.coords, id, g);
                    for (int b = 0; b < 4; ++b) {
                        const int s = kuhn_slot(lv[b][0] - i, lv[b][1] - j, lv[b][2] - k);
                        if (s < 0) continue;   // not reached: the vertices of a Kuhn tet are Kuhn neighbours
                        row[s] += vol * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]);
                    }
                    touched = true;
                }
            }
    double *A = F.A + ((long long)y * F.nv + v) * MG_SLOTS;
    for (int s = 0; s < MG_SLOTS; ++s) A[s] = row[s];
    int fl = V_OFF;
    if (touched) {
        const int d = F.axis[y];
        const int c = d == 0 ? i : (d == 1 ? j : k);
        fl = c == 0 ? V_INLET : (c == n ? V_OUTLET : V_FREE);
    }
    F.flag[(long long)y * F.nv + v] = fl;
}

__device__ inline double block_sum(double v, double *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += red[k];
    return s;
}

// (A x)_v over the stencil; neighbours outside the lattice carry zero coefficients.
__device__ inline double stencil_apply(const double *A, const double *x, long long v, int n) {
    const int i = (int)(v % (n + 1)), j = (int)((v / (n + 1)) % (n + 1)), k = (int)(v / ((long long)(n + 1) * (n + 1)));
    double s = 0.0;
    for (int t = 0; t < MG_SLOTS; ++t) {
        const double a = A[t];
        if (a == 0.0) continue;
        int dx, dy, dz;
        kuhn_offset(t, dx, dy, dz);
        s += a * x[vid(i + dx, j + dy, k + dz, n)];
    }
    return s;
}

// Jacobi-preconditioned CG for yarn blockIdx.x: free vertices unknown, inlet 0,
// outlet 1, vertices off the yarn excluded.  Stops when r.z <= rtol^2 r0.z0.
__global__ __launch_bounds__(FLOW_BS) void flow_cg_kernel(FlowArgs F, double rtol2, int max_iter) {
    __shared__ double red[FLOW_BS / 64];
    const int y = blockIdx.x, n = F.n;
    const long long nv = F.nv, base = (long long)y * nv;
    const double *A = F.A + base * MG_SLOTS;
    const int *fl = F.flag + base;
    double *phi = F.phi + base, *r = F.r + base, *p = F.p + base, *q = F.q + base;
    for (long long v = threadIdx.x; v < nv; v += blockDim.x) {
        phi[v] = fl[v] == V_OUTLET ? 1.0 : 0.0;
        p[v] = 0.0;
    }
    __syncthreads();
    double loc = 0.0;
    for (long long v = threadIdx.x; v < nv; v += blockDim.x) {
        double rv = 0.0;
        if (fl[v] == V_FREE) rv = -stencil_apply(A + v * MG_SLOTS, phi, v, n);
        r[v] = rv;
        const double z = fl[v] == V_FREE ? rv / A[v * MG_SLOTS] : 0.0;
        p[v] = z;
        loc += rv * z;
    }
    double rz = block_sum(loc, red);
    const double rz0 = rz;
    int it = 0;
    bool conv = rz <= rtol2 * rz0 || rz == 0.0;
    while (!conv && it < max_iter) {
        loc = 0.0;
        for (long long v = threadIdx.x; v < nv; v += blockDim.x) {
            double qv = 0.0;
            if (fl[v] == V_FREE) qv = stencil_apply(A + v * MG_SLOTS, p, v, n);
            q[v] = qv;
            loc += p[v] * qv;
        }
        const double pq = block_sum(loc, red);
        if (!(pq > 0.0)) break;
        const double alpha = rz / pq;
        loc = 0.0;
        for (long long v = threadIdx.x; v < nv; v += blockDim.x) {
            if (fl[v] != V_FREE) continue;
            phi[v] += alpha * p[v];
            const double rv = r[v] - alpha * q[v];
            r[v] = rv;
            loc += rv * rv / A[v * MG_SLOTS];
        }
        const double rzn = block_sum(loc, red);
        ++it;
        conv = rzn <= rtol2 * rz0;
        const double beta = rzn / rz;
        rz = rzn;
        for (long long v = threadIdx.x; v < nv; v += blockDim.x)
            if (fl[v] == V_FREE) p[v] = r[v] / A[v * MG_SLOTS] + beta * p[v];
        __syncthreads();
    }
    if (threadIdx.x == 0) F.iters[y] = conv ? it : -(it + 1);
}

// Fibre axis of every tet: normalised gradient of its yarn's potential; zero for matrix tets.
__global__ __launch_bounds__(256) void flow_axis_kernel(FlowArgs F, int nyarn, double *axis, int *bad) {
    const int n = F.n;
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= 6LL * n * n * n) return;
    const int y = F.phase[e] - 1;
    double out[3] = {0.0, 0.0, 0.0};
    if (y >= 0 && y < nyarn) {
        const int t = (int)(e % 6);
        const long long cell = e / 6;
        const int ci = (int)(cell % n), cj = (int)((cell / n) % n), ck = (int)(cell / ((long long)n * n));
        int lv[4][3];
        tet_lattice(ci, cj, ck, t, lv);
        long long id[4];
        for (int a = 0; a < 4; ++a) id[a] = vid(lv[a][0], lv[a][1], lv[a][2], n);
        double g[4][3];
        tet_grads(F.coords, id, g);
        const double *phi = F.phi + (long long)y * F.nv;
        for (int a = 0; a < 4; ++a)
            for (int d = 0; d < 3; ++d) out[d] += phi[id[a]] * g[a][d];
        const double nr = sqrt(out[0] * out[0] + out[1] * out[1] + out[2] * out[2]);
        if (nr > 0.0) {
            for (int d = 0; d < 3; ++d) out[d] /= nr;
        } else {
            atomicOr(bad, 1);
        }
    }
    for (int d = 0; d < 3; ++d) axis[3 * e + d] = out[d];
}

}  // namespace
}  // namespace chom

using namespace chom;

extern "C" int chom_yarn_directions(const chom_mesh *mesh, int32_t n_yarns, const int32_t *yarn_axis, double rtol,
                                    int32_t max_iter, double *fibre_axis, void *hip_stream) {
    if (!mesh || !yarn_axis || !fibre_axis || n_yarns < 1 || n_yarns > 127 || !(rtol > 0.0) || max_iter < 1 ||
        !mesh->coords || !mesh->tets || !mesh->phase) {
        set_error("chom_yarn_directions: null argument, n_yarns outside 1..127, rtol <= 0 or max_iter < 1");
        return CHOM_EINVAL;
    }
    for (int y = 0; y < n_yarns; ++y)
        if (yarn_axis[y] < 0 || yarn_axis[y] > 2) {
            set_error("chom_yarn_directions: yarn_axis entries must be 0, 1 or 2");
            return CHOM_EINVAL;
        }
    const int n = (int)std::lround(std::cbrt((double)mesh->n_tets / 6.0));
    if (n < 1 || 6LL * n * n * n != mesh->n_tets || (long long)(n + 1) * (n + 1) * (n + 1) != mesh->n_vertices) {
        set_error("chom_yarn_directions: mesh is not a Kuhn lattice (need (n+1)^3 vertices and 6 n^3 tets)");
        return CHOM_EMESH;
    }
    const long long nv = mesh->n_vertices, nt = mesh->n_tets;
    hipStream_t s = (hipStream_t)hip_stream;
    // the kernels take the lattice connectivity: check that the mesh has it
    std::vector<int32_t> ht(4 * nt);
    std::vector<int8_t> hph(nt);
    if (mesh->on_device) {
        CHOM_HIP(hipMemcpy(ht.data(), mesh->tets, sizeof(int32_t) * 4 * nt, hipMemcpyDeviceToHost));
        CHOM_HIP(hipMemcpy(hph.data(), mesh->phase, nt, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(ht.data(), mesh->tets, sizeof(int32_t) * 4 * nt);
        std::memcpy(hph.data(), mesh->phase, nt);
    }
    for (long long e = 0; e < nt; ++e) {
        const int t = (int)(e % 6);
        const long long cell = e / 6;
        const int ci = (int)(cell % n), cj = (int)((cell / n) % n), ck = (int)(cell / ((long long)n * n));
        int p0, p1;
        kuhn_perm(t, p0, p1);
        int v[4][3] = {{ci, cj, ck}, {ci, cj, ck}, {ci, cj, ck}, {ci + 1, cj + 1, ck + 1}};
        v[1][p0] += 1;
        v[2][p0] += 1;
        v[2][p1] += 1;
        long long want[4], got[4];
        for (int a = 0; a < 4; ++a) {
            want[a] = v[a][0] + (long long)(n + 1) * (v[a][1] + (long long)(n + 1) * v[a][2]);
            got[a] = ht[4 * e + a];
        }
        std::sort(want, want + 4);
        std::sort(got, got + 4);
        for (int a = 0; a < 4; ++a)
            if (want[a] != got[a]) {
                set_error("chom_yarn_directions: tet " + std::to_string(e) + " does not match the Kuhn lattice");
                return CHOM_EMESH;
            }
        if (hph[e] < 0 || hph[e] > n_yarns) {
            set_error("chom_yarn_directions: phase outside 0..n_yarns");
            return CHOM_EMESH;
        }
    }
    DevBuf<double> dc, dA, dphi, dr, dp, dq, dax;
    DevBuf<int8_t> dph;
    DevBuf<int> dflag, daxis, diters, dbad;
    CHOM_HIP(dc.ensure(3 * nv));
    CHOM_HIP(dph.ensure(nt));
    CHOM_HIP(daxis.ensure(n_yarns));
    CHOM_HIP(dA.ensure((size_t)n_yarns * nv * MG_SLOTS));
    CHOM_HIP(dflag.ensure((size_t)n_yarns * nv));
    for (DevBuf<double> *b : {&dphi, &dr, &dp, &dq}) CHOM_HIP(b->ensure((size_t)n_yarns * nv));
    CHOM_HIP(diters.ensure(n_yarns));
    CHOM_HIP(dbad.ensure(1));
    const hipMemcpyKind kind = mesh->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    CHOM_HIP(hipMemcpyAsync(dc.p, mesh->coords, sizeof(double) * 3 * nv, kind, s));
    CHOM_HIP(hipMemcpyAsync(dph.p, hph.data(), nt, hipMemcpyHostToDevice, s));
    CHOM_HIP(hipMemcpyAsync(daxis.p, yarn_axis, sizeof(int) * n_yarns, hipMemcpyHostToDevice, s));
    CHOM_HIP(hipMemsetAsync(dbad.p, 0, sizeof(int), s));
    FlowArgs F;
    F.n = n;
    F.nv = nv;
    F.coords = dc.p;
    F.phase = dph.p;
    F.axis = daxis.p;
    F.A = dA.p;
    F.flag = dflag.p;
    F.phi = dphi.p;
    F.r = dr.p;
    F.p = dp.p;
    F.q = dq.p;
    F.iters = diters.p;
    flow_assemble_kernel<<<dim3((unsigned)((nv + 255) / 256), n_yarns), 256, 0, s>>>(F);
    CHOM_HIP(hipGetLastError());
    flow_cg_kernel<<<n_yarns, FLOW_BS, 0, s>>>(F, rtol * rtol, max_iter);
    CHOM_HIP(hipGetLastError());
    double *out = fibre_axis;
    if (!mesh->on_device) {
        CHOM_HIP(dax.ensure(3 * nt));
        out = dax.p;
    }
    flow_axis_kernel<<<(unsigned)((nt + 255) / 256), 256, 0, s>>>(F, n_yarns, out, dbad.p);
    CHOM_HIP(hipGetLastError());
    std::vector<int> its(n_yarns);
    int hbad = 0;
    CHOM_HIP(hipMemcpyAsync(its.data(), diters.p, sizeof(int) * n_yarns, hipMemcpyDeviceToHost, s));
    CHOM_HIP(hipMemcpyAsync(&hbad, dbad.p, sizeof(int), hipMemcpyDeviceToHost, s));
    if (!mesh->on_device) CHOM_HIP(hipMemcpyAsync(fibre_axis, out, sizeof(double) * 3 * nt, hipMemcpyDeviceToHost, s));
    CHOM_HIP(hipStreamSynchronize(s));
    for (int y = 0; y < n_yarns; ++y) {
        bool has = false;
        for (long long e = 0; e < nt && !has; ++e) has = hph[e] == y + 1;
        if (!has) continue;
        if (its[y] < 0) {
            set_error("chom_yarn_directions: the potential of yarn " + std::to_string(y + 1) +
                      " did not converge in max_iter steps (directions written)");
            return CHOM_ENOCONV;
        }
    }
    if (hbad) {
        set_error("chom_yarn_directions: a yarn tet has no potential gradient (a yarn part that does not reach "
                  "its inlet or outlet face)");
        return CHOM_EMESH;
    }
    return CHOM_OK;
}
