// Host-side internal interfaces of libchom (kernel launchers, workspaces).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "chom.h"
#include "common.h"

namespace chom {

// Per-column (problem x load case) solver state, device-resident.
struct ColState {
    double alpha, beta, rz, rz_init, eref, pq, rz_prev, pad;
    int done;    // 0 active, 1 converged, 2 breakdown / no progress
    int iters;
    int pad2[2];
};

// Vector-kernel launch shape: blocks per problem along x, problems along y.
constexpr int VEC_BS = 256;
constexpr int FIN_BS = 64;

// Partial-sum record sizes (doubles per load case).
__host__ __device__ inline int upd_rec(int C, int nrow) { return 2 + C * nrow; }

// ------------------------------------------------------------------ launchers
hipError_t launch_generate(int n, double *coords, int32_t *tets, int8_t *phase, double *axis,
                           hipStream_t s);

// Element data: fibre axis + phase (both precisions) and, for distorted grids,
// per-tet geometry.  Inputs are device arrays of the mesh.
hipError_t launch_element_setup(const Geo &G, const double *coords, const int32_t *tets_sorted,
                                const int8_t *phase, const double *axis, double4 *elem64,
                                float4 *elem32, double *geo64, float *geo32, int *bad_count,
                                hipStream_t s);
hipError_t launch_rows(const Geo &G, double *rows, hipStream_t s);

// Diagonal blocks (FP64 accumulation) and their inverses for a class of problems.
template <int C>
hipError_t launch_precond(const Geo &G, const Prob *probs, int nprob, double *diag,
                          double *minv64, float *minv32, hipStream_t s);
template <int C>
hipError_t launch_gram(const Geo &G, int nprob, const double *minv64, const float *minv32,
                       double *gram_partial, int nwg, double *ginv64, double *ginv32, int *bad,
                       hipStream_t s);
template <int C, int R>
hipError_t launch_rhs(const Geo &G, const Prob *probs, int nprob, long long vals_per_prob,
                      double *b, ColState *cols, hipStream_t s);

// Operator y = K x (q zeroed by the caller), fused element energies x.K.x per column.
template <typename T, int C, int R>
hipError_t launch_operator(const Geo &G, const Prob *probs, int nprob, const T *x, T *y,
                           double *partial_pq, const int *prob_active, hipStream_t s);
int operator_tiles(const Geo &G);

// CG vector kernels.
template <typename T, int C, int R>
hipError_t launch_cg_init(const Geo &G, int nprob, long long vpp, const T *b, T *x, T *r, T *z,
                          const void *minv, double *partial, int nwg, hipStream_t s);
template <typename T, int C, int R>
hipError_t launch_cg_dir(const Geo &G, int nprob, long long vpp, T *r, const T *z, T *p, T *q,
                         const void *minv, const double *ycoef, const ColState *cols,
                         const int *prob_active, int nwg, hipStream_t s);
template <typename T, int C, int R>
hipError_t launch_cg_update(const Geo &G, int nprob, long long vpp, T *x, T *r, T *z, const T *p,
                            const T *q, const void *minv, const ColState *cols, double *partial,
                            const int *prob_active, int nwg, hipStream_t s);
template <int C, int R>
hipError_t launch_finish_alpha(int nprob, const double *partial_pq, int nparts, ColState *cols,
                               hipStream_t s);
template <int C, int R>
hipError_t launch_finish_beta(int nprob, int nrow, const double *partial, int nparts,
                              const double *ginv, double *ycoef, ColState *cols, int *prob_active,
                              int first, double rtol2, int use_init, hipStream_t s);

template <int C, int R>
hipError_t launch_finish_beta_masked(int nprob, int nrow, const double *partial, int nparts,
                                     const double *ginv, double *ycoef, ColState *cols,
                                     int *prob_active, double rtol2, const ColState *mask,
                                     hipStream_t s);

// Refinement helpers (FP64 outer vectors).
template <int C, int R>
hipError_t launch_residual64(const Geo &G, int nprob, long long vpp, const double *b,
                             const double *q64, double *r64, float *r32, hipStream_t s);
template <int C, int R>
hipError_t launch_proj_resid(const Geo &G, int nprob, long long vpp, double *r64, float *r32,
                             const double *minv64, const double *ycoef, double *partial, int nwg,
                             hipStream_t s);
template <int C, int R>
hipError_t launch_axpy_x64(int nprob, long long vpp, double *x64, const float *d32, hipStream_t s);
template <int C, int R>
hipError_t launch_project(const Geo &G, int nprob, long long vpp, double *x64, const double *minv64,
                          const double *ginv64, double *partial, int nwg, hipStream_t s);

// Homogenisation average: partial sums per block, reduced by the finish kernel.
template <int C, int R>
hipError_t launch_average(const Geo &G, const Prob *probs, int nprob, long long vpp,
                          const double *x64, double *partial, int nwg, double *out,
                          hipStream_t s);

// Error handling helpers (api.cpp).
void set_error(const std::string &msg);

}  // namespace chom
