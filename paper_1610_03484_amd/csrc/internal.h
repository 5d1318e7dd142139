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
// done: COL_ACTIVE, or why the column stopped (any nonzero value stops it).
enum { COL_ACTIVE = 0, COL_CONVERGED = 1, COL_BREAKDOWN = 2, COL_NONFINITE = 3, COL_CAPPED = 4 };
struct ColState {
    double alpha, beta, rz, rz_init, eref, pq, rz_prev;
    double energy;   // running estimate of (x_lin + u)^T K (x_lin + u): eref minus alpha r.z of every CG step
    int done;    // COL_* above
    int iters;   // CG steps taken by this column (all solves of the call)
    int iters0;  // iters at the start of the current solve (the cap counts from here)
    int pad2;
};

constexpr int FIN_BS = 64;

// Shape of one class launch (all problems of one physics in a batch).
struct Launch {
    const Geo *geos;      // device array of RVE geometries
    const Prob *probs;    // device array of problems
    int nprob;
    int nwg;              // vector-kernel workgroups per problem
    int max_tiles;        // largest operator tile count among the problems
    int nr;               // largest constraint row count among the problems (0, 1, 4)
    int rg;               // load cases per operator workgroup
    long long max_tets;   // largest tet count among the problems
    int order;            // polynomial order of every problem of the class
    long long total_q;    // values of the operator output of the class
    const double *ef64;   // orders 3, 4: element factors Q_e (packed symmetric 3C x 3C), per problem at Prob.eoff
    const float *ef32;
    // two-level preconditioner (mg.hip); on = 0: block Jacobi alone
    struct Mg {
        int on;
        int nlev;                  // largest level count among the problems
        int nwg[MG_MAXLEV];        // workgroups per problem of the level-l kernels
        int sweeps;                // l1 block-Jacobi sweeps on the coarsest level
        long long total_pts;       // coarse points of the class
        double *A64, *D64;         // FP64 stencils and l1 inverses (setup)
        const void *A, *Dinv;      // the same in the precision of the solve
        void *r, *xp, *res, *x;    // level vectors [moff * R * C][R][mg_pts][C]
        double *rows1;             // level-1 restricted constraint rows [points][4]
        long long max_pts[MG_MAXLEV];  // largest level-l point count of the class
        long long lds_elems;       // LDS of the fused kernel (elements of the solve precision)
        int lds_vec, lds_sten;     // levels >= 2 vectors / coarsest stencils in LDS
        long long small_elems;     // > 0: FP32 levels >= 2 small enough for mg_fused_small_kernel (its LDS, floats)
        int small_bs;              // its threads (256 or 512: at least the points of the largest owned level)
        void *W;                   // coarse part of B C^T [moff + vertex][4C][C]
    } mg;
};

// ------------------------------------------------------------------ launchers
hipError_t launch_generate(int n, double *coords, int32_t *tets, int8_t *phase, double *axis, hipStream_t s);

// Per RVE (geometry by value): element data and, for distorted grids, per-tet geometry.
hipError_t launch_element_setup(const Geo &G, const double *coords, const int32_t *tets_sorted,
                                const int8_t *phase, const double *axis, double4 *elem64, float4 *elem32,
                                double *geo64, float *geo32, int *bad_count, hipStream_t s);
hipError_t launch_rows(const Geo &G, double *rows, hipStream_t s);
int operator_tiles(const Geo &G);

// Per class of problems.
template <int C>
hipError_t launch_precond(const Launch &L, long long total_pts, double *diag, double *minv64, float *minv32,
                          double *qscratch, hipStream_t s);
template <int C>
hipError_t launch_gram(const Launch &L, const double *minv64, const float *minv32, double *gram_partial, int nwg,
                       double *ginv64, double *ginv32, int *bad, hipStream_t s, double *gmat = nullptr);
// Load vectors b and linear-field energies (cols[].eref); q64t: FP64 tile-box
// scratch, acc_pq: accumulator scratch (both overwritten).
template <int C, int R>
hipError_t launch_rhs(const Launch &L, long long total_vals, double *b, ColState *cols, double *q64t,
                      double *acc_pq, hipStream_t s);
template <int C, int R>
hipError_t launch_rhs_operator(const Launch &L, int rg, double *y, double *acc_pq, hipStream_t s);
// Tile boxes of the order-2 diagonal point blocks (group 0 of the FP64 boxes;
// packed xx yy zz xy yz xz for elasticity); summed per point by launch_precond.
template <int C, int R> hipError_t launch_diag_operator(const Launch &L, double *y, hipStream_t s);

template <typename T, int C, int R>
hipError_t launch_operator(const Launch &L, int nprob, int rg, const T *x, T *y,
                           double *partial_pq, const int *prob_active, hipStream_t s);

template <typename T, int C, int R>
hipError_t launch_cg_init(const Launch &L, const T *b, T *x, T *r, const void *minv, double *accbuf, hipStream_t s);
// Direction step; also applies the previous step's x += alpha p (deferred from
// the update kernel); launch_cg_flush_x applies the last one after a solve.
template <typename T, int C, int R>
hipError_t launch_cg_dir(const Launch &L, T *x, T *r, T *p, const void *minv, const double *ycoef,
                         const ColState *cols, const int *prob_active, hipStream_t s,
                         const void *mg_x0 = nullptr, const void *mg_W = nullptr);
template <typename T, int C, int R>
hipError_t launch_cg_update(const Launch &L, T *r, const T *q, const void *minv, const ColState *cols,
                            double *accbuf, const int *prob_active, hipStream_t s);
template <typename T, int C, int R>
hipError_t launch_cg_flush_x(const Launch &L, T *x, const T *p, const ColState *cols, hipStream_t s);
template <int C, int R>
hipError_t launch_finish_alpha(const Launch &L, double *acc_pq, ColState *cols, hipStream_t s);
template <int C, int R>
hipError_t launch_finish_beta(const Launch &L, double *accbuf, const double *ginv, double *ycoef, ColState *cols,
                              int *prob_active, int first, double rtol2, int use_init, const ColState *mask,
                              hipStream_t s, int max_iter = 0, const ColState *esrc = nullptr, double loose = 0.0);
template <int C, int R>
hipError_t launch_proj_resid(const Launch &L, double *r64, float *r32, const double *minv64,
                             const double *ycoef, double *partial, hipStream_t s);
template <int C, int R>
hipError_t launch_residual64(const Launch &L, const double *b, const double *q64t, double *r64, float *r32,
                             hipStream_t s);
hipError_t launch_axpy_x64(long long total, double *x64, const float *d32, hipStream_t s);
hipError_t launch_axpy64(long long total, double *x64, const double *d64, hipStream_t s);
// Clears n doubles with a kernel (safe inside captured graphs).
hipError_t launch_zero(double *p, long long n, hipStream_t s);
template <int C, int R>
hipError_t launch_project(const Launch &L, double *x64, const double *minv64, const double *ginv64,
                          double *partial, hipStream_t s);
// out: energy form of the averages [prob][NC][R]; corr (nullable, with r64):
// the residual term (1/V) u_i . r_j that separates it from the plain average.
template <int C, int R>
hipError_t launch_average(const Launch &L, const double *x64, const double *r64, double *partial, int nwg,
                          double *out, hipStream_t s, double *corr = nullptr);

void set_error(const std::string &msg);

// ------------------------------------------------------------------ two-level preconditioner (mg.hip)
// Fills G.mg_*: level 0 is the vertex lattice of the n^3 grid; a level is
// halved while its cell count is even and the half is at least 3 (so periodic
// neighbours never alias).  No hierarchy (mg_nlev = 0) unless there are at least
// two levels (n even, n >= 6).
void mg_levels(Geo &G);
// Host index tables of the coarse levels (see Geo.mg_nbr / mg_child / mg_par),
// [mg_pts][16] ints each.
void mg_tables(const Geo &G, std::vector<int> &nbr, std::vector<int> &child, std::vector<int> &par);
// Stencils of every level (FP64), their l1 inverses, and the copies in T.
template <typename T, int C> hipError_t launch_mg_stencils(const Launch &L, T *A, T *Dinv, hipStream_t s);
// One V-cycle on the fine vectors r (all load cases), from the n/2 grid: output
// e_1 in the level-1 block of L.mg.x; with `accbuf`, r . Q e_1 and C Q e_1 are
// added to the CG step's accumulators.
template <typename T, int C, int R>
hipError_t launch_mg_vcycle(const Launch &L, const T *r, double *accbuf, const int *prob_active, hipStream_t s);
// Coarse correction f = e_1 - W y of the current CG step (into the level-1 res block).
template <typename T, int C, int R>
hipError_t launch_mg_fcorr(const Launch &L, const double *ycoef, const int *prob_active, hipStream_t s);
// W = V P^T C^T (constraint columns, in batches of R) using `tmp` (a fine
// vector), then the Gram matrix C B C^T = gmat + C P W and its inverse.
template <typename T, int C, int R>
hipError_t launch_mg_gram(const Launch &L, T *tmp, const double *gmat, double *partial, int nwg, double *ginv,
                          int *bad, hipStream_t s);

// orders 3, 4 (hp.hip)
hipError_t launch_rows_hp(const Geo &G, double *rows, hipStream_t s);
template <int C> hipError_t launch_diag_hp(const Launch &L, double *diag, hipStream_t s);
template <int C, int R> hipError_t launch_rhs_hp(const Launch &L, double *b, ColState *cols, hipStream_t s);
template <int C, int R>
hipError_t launch_average_partial_hp(const Launch &L, const double *x64, double *partial, int nwg, hipStream_t s);
template <int C> hipError_t launch_factors_hp(const Launch &L, double *ef64, float *ef32, hipStream_t s);
template <typename T, int C, int R>
hipError_t launch_operator_hp(const Launch &L, int nprob, int rg, const T *x, T *y, double *partial_pq,
                              const int *prob_active, hipStream_t s);

// Homogenises `batch` records given in host memory with the RVE's own batch
// workspace, whatever the RVE's pointer convention (outputs in host memory too).
int rve_homogenise_host(chom_rve *rve, const chom_params *params, int batch, double *C, double *K, double *D,
                        chom_report *rep);
void rve_settings(const chom_rve *rve, double *c_sat, int *degrade_yarn);
// Surrogate gradient evaluation in a caller-provided device workspace (mlp_api.cpp).
int mlp_loss_grad_ws(chom_mlp *m, int member, const double *p, const double *c, const double *k, const double *d,
                     long long n, double *loss, float *grad, unsigned char *ws, long long max_rows);
bool mlp_ready(const chom_mlp *m, int member);
// Yarn tags of any tet mesh of the unit cube (mesh.hip).
hipError_t launch_tag(long long nt, const double *coords, const int32_t *tets, int8_t *phase, double *axis,
                      hipStream_t s);
// 1 if the ensemble's bulk arrays are device pointers (chom_mlp_options.device_ptrs).
int mlp_device_ptrs(const chom_mlp *m);

#define CHOM_HIP(...)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (__VA_ARGS__);                                                         \
        if (e_ != hipSuccess) {                                                                \
            set_error(std::string("HIP error: ") + hipGetErrorString(e_) + " at " #__VA_ARGS__); \
            return e_ == hipErrorOutOfMemory ? CHOM_ENOMEM : CHOM_EDEVICE;                     \
        }                                                                                      \
    } while (0)

#define CHOM_TRY(...)                    \
    do {                                 \
        int st_ = (__VA_ARGS__);         \
        if (st_ != CHOM_OK) return st_;  \
    } while (0)

// Pinned host buffer owned by a handle (device-to-host polls copy into it
// directly, without a staging copy).
template <typename T> struct HostBuf {
    T *p = nullptr;
    size_t n = 0;
    HostBuf() = default;
    HostBuf(const HostBuf &) = delete;
    HostBuf &operator=(const HostBuf &) = delete;
    ~HostBuf() { release(); }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
    }
    hipError_t ensure(size_t count) {
        if (count <= n && p) return hipSuccess;
        release();
        if (count == 0) count = 1;
        hipError_t e = hipHostMalloc((void **)&p, sizeof(T) * count, hipHostMallocDefault);
        if (e == hipSuccess) n = count;
        return e;
    }
};

// Device buffer owned by a handle.
template <typename T> struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    hipError_t ensure(size_t count) {
        if (count <= n && p) return hipSuccess;
        release();
        if (count == 0) count = 1;
        hipError_t e = hipMalloc((void **)&p, sizeof(T) * count);
        if (e == hipSuccess) n = count;
        return e;
    }
};


}  // namespace chom
