/*
 * chom.h -- C ABI of the MI355X RVE computational-homogenisation library.
 *
 * The library computes, for a representative volume element (RVE) of a
 * plain-weave composite, the homogenised stiffness C_bar (6x6), conductivity
 * K_bar (3x3) and diffusivity D_bar (3x3) of first-order computational
 * homogenisation (paper Sec. 2): for each unit macro strain (6 load cases,
 * Eq. Eq_C_stress) and each unit macro gradient of temperature and moisture
 * (3 + 3 load cases, Eqs. eq_RVE_disc_Eqs_field, eq_homo_flux) it solves the
 * micro equilibrium problem (Eq. RVE_Eq_var_final) on the RVE under linear
 * Dirichlet, periodic or uniform-traction (Neumann) constraints (Sec. 2,
 * items 1-3; Eqs. eq_RVE_disc_Eqs, eq_mat_C_and_D) and volume-averages the
 * micro stress / flux (Eq. macro_stress).  Matrix stiffness is degraded with
 * the temperature-moisture-time law of Sec. 4 (Eq. Eq_Model_final1), applied
 * to the matrix only (Sec. 5).
 *
 * Conventions
 *   - Every function returns an int status (CHOM_OK = 0 or a negative code).
 *     No exception crosses the ABI.  chom_last_error() gives a message for the
 *     last failing call on the calling thread.
 *   - Voigt order [11, 22, 33, 12, 23, 31], strains with engineering shear
 *     (paper Sec. 2, definition of the macro-strain vector); stresses without.
 *   - C_hom is returned as its 21 upper-triangle entries, row-major
 *     (C[0][0], C[0][1], ..., C[0][5], C[1][1], ...), where column j of the
 *     unsymmetrised C_bar is the homogenised stress of unit strain j.
 *     K_hom and D_hom are returned as [xx, yy, zz, xy, yz, xz] of the upper
 *     triangle.  Units pass through (moduli in the units of the inputs).
 *   - Inputs are borrowed for the duration of the call and copied; handles are
 *     owned by the caller and released with the matching *_destroy.  Output
 *     buffers are allocated by the caller.
 *   - Pointers are host pointers unless a flag says they are device pointers
 *     (chom_mesh.on_device, chom_options.device_ptrs).  Device pointers must be
 *     on the current HIP device.  Work is queued on chom_options.hip_stream (or
 *     the null stream); chom_homogenise returns after the results are written.
 */
#ifndef CHOM_H
#define CHOM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
enum {
    CHOM_OK = 0,
    CHOM_EINVAL = -1,     /* bad argument (null pointer, size, option)            */
    CHOM_EMESH = -2,      /* mesh not a supported lattice, or degenerate tet       */
    CHOM_EMATERIAL = -3,  /* material not positive definite after factors/damage  */
    CHOM_ENOCONV = -4,    /* results written, some load case did not converge     */
    CHOM_EDEVICE = -5,    /* HIP runtime error or no device                        */
    CHOM_ENOMEM = -6      /* device allocation failed                              */
};

enum { CHOM_BC_DIRICHLET = 0, CHOM_BC_PERIODIC = 1, CHOM_BC_NEUMANN = 2 };
enum { CHOM_FP64 = 0, CHOM_FP32_REFINED = 1 };
/* Preconditioners of the CG solves (the paper factorises directly, Sec. 2):
 * CHOM_PRECOND_BLOCK_JACOBI: the inverse point blocks M^-1 of K.
 * CHOM_PRECOND_TWO_LEVEL: M^-1 + P V P^T, with P the injection of the vertex
 *   (P1) values -- the vertex functions of the hierarchic basis are the P1 hats,
 *   so P^T K P is the P1 stiffness -- and V one symmetric V-cycle on the P1
 *   spaces of the Kuhn grids with n, n/2, ... cells (Galerkin coarse matrices,
 *   l1 block-Jacobi smoothing).  RVEs with odd n or n < 6 have no coarse grid
 *   and take block Jacobi alone. */
enum { CHOM_PRECOND_BLOCK_JACOBI = 0, CHOM_PRECOND_TWO_LEVEL = 1 };

typedef struct chom_rve chom_rve;
typedef struct chom_batch chom_batch;
typedef struct chom_mlp chom_mlp;   /* learned surrogate ensemble (below) */

/* RVE mesh.  Supported meshes: the Kuhn split of an n x n x n cell grid of the
 * box [lo, hi] -- (n+1)^3 vertices numbered i + (n+1)(j + (n+1)k), 6 n^3 tets,
 * cell-major, the six tets of a cell in the axis-permutation order
 * (0,1,2),(0,2,1),(1,0,2),(1,2,0),(2,0,1),(2,1,0), each tet
 * (v0, v0+e_a, v0+e_a+e_b, v0+(1,1,1)) in any vertex order.  Vertex
 * coordinates may be moved (distorted meshes) as long as every tet keeps the
 * orientation of its undistorted shape and boundary vertices stay on their
 * faces; periodic BCs additionally need matching opposite faces.  Other meshes
 * are rejected with CHOM_EMESH.
 * phase: 0 = matrix, 1..4 = yarn; fibre_axis: unit vector per tet (ignored
 * for matrix tets). */
typedef struct {
    int32_t n_vertices;
    int32_t n_tets;
    const double *coords;      /* [n_vertices][3]                        */
    const int32_t *tets;       /* [n_tets][4]                            */
    const int8_t *phase;       /* [n_tets]                               */
    const double *fibre_axis;  /* [n_tets][3]                            */
    double lo[3], hi[3];
    int32_t on_device;         /* 1: the four arrays are device pointers */
} chom_mesh;

/* Base constituent properties.  Matrix: isotropic (E, nu), conductivity k,
 * diffusivity D.  Yarn: transversely isotropic about the fibre axis: E1 along
 * the fibre, E2 = E3 across, G12 = G13, major Poisson ratio nu12
 * (S12 = -nu12/E1), nu23 with G23 = E2 / (2 (1 + nu23)); conductivity and
 * diffusivity k1, D1 along and k2, D2 across the fibre. */
typedef struct {
    double E, nu, k, D;
    double E1, E2, G12, nu12, nu23, k1, k2, D1, D2;
} chom_materials;

/* One macro Gauss point: exposure temperature (deg C), moisture (wt%),
 * exposure time (years) and eight property factors multiplying the groups
 * matrix {E}, {nu}, {k}, {D}, yarn {E1, E2, G12}, {nu12, nu23}, {k1, k2},
 * {D1, D2}.  The matrix modulus is further multiplied by
 * (1 - omega) = exp(-gamma(c) alpha(T) t): alpha(T) = beta ln(1 - T/T_g) with
 * absolute temperatures, beta = -0.001682 per day, T_g = 126 C (Sec. 4, Eqs.
 * Eq_alphaT, Eq_alphaT_LSF), gamma(c) = c / c_sat (Eq. Eq_Model3), t in days
 * (365.25 per year). */
typedef struct {
    double T_celsius, c_wt, t_years, factor[8];
} chom_params;

typedef struct {
    int32_t precision;     /* CHOM_FP64 or CHOM_FP32_REFINED                           */
    int32_t precond;       /* CHOM_PRECOND_BLOCK_JACOBI or CHOM_PRECOND_TWO_LEVEL      */
    int32_t max_iter;      /* CG iteration cap per solve (per inner solve when refined) */
    int32_t max_refine;    /* refinement steps cap (CHOM_FP32_REFINED)                 */
    double rtol;           /* stop a load case when r.P r <= rtol^2 E: P the
                              preconditioner (M^-1, or the two-level B), r the projected
                              residual (the FP64 one of the refinement), E the load
                              case's energy (x_lin + u)^T K (x_lin + u), tracked from the
                              CG steps and kept within [1e-6, 1] x the linear-field
                              energy x_lin^T K x_lin.  Relative to E, the energy-form
                              averages are accurate against the homogenised value itself,
                              also in the soft directions of a degraded matrix; past a
                              yarn/matrix shear-modulus ratio of 3e4 ((1 - omega) below
                              about 1e-4) the mechanical tests use rtol^2 x 3e4 / ratio,
                              which keeps the energy-weighted error of C_bar at rtol 3e-5
                              near 1e-9 at (1 - omega) = 1e-6 and 6e-7 at 1e-8 (0.1
                              without it)                                                */
    double inner_rtol;     /* FP32 inner solves: stop when r.B r falls below
                              inner_rtol^2 times the smaller of its initial value and E */
    double c_sat;          /* moisture content (wt%) with gamma = 1                    */
    int32_t degrade_yarn;  /* 1: the damage factor also scales the yarn moduli         */
    int32_t device_ptrs;   /* 1: params and outputs of chom_homogenise are on device  */
    void *hip_stream;      /* hipStream_t to queue work on (NULL: null stream)        */
} chom_options;

/* Why a load case did not converge (chom_report.fail). */
enum {
    CHOM_FAIL_NONE = 0,       /* converged                                                   */
    CHOM_FAIL_CAP = 1,        /* max_iter CG steps (or max_refine refinement steps) reached   */
    CHOM_FAIL_BREAKDOWN = 2,  /* p.Kp <= 0 (operator not positive definite in that direction) */
    CHOM_FAIL_NONFINITE = 3   /* a CG scalar became NaN or infinite; the solve stopped there   */
};

typedef struct {
    int32_t iters[12];        /* CG iterations per load case: 6 mech, 3 thermal, 3 moisture */
    int32_t refine_steps[3];  /* refinement steps (mech, thermal, moisture)                 */
    int32_t status;           /* CHOM_OK or CHOM_ENOCONV                                    */
    double resid[12];         /* final sqrt(r.P r / linear-field energy) per load case (P as
                                 for chom_options.rtol; 0 when the projected r.P r fell to
                                 the rounding level of the unprojected one)                  */
    double asym;              /* ||C - C^T||_F / ||C||_F of the unsymmetrised C_bar           */
    double omega_keep;        /* (1 - omega) applied to the matrix modulus                   */
    int32_t fail[12];         /* CHOM_FAIL_* per load case                                   */
    int32_t fp64_fallback[3]; /* CHOM_FP32_REFINED: 1 if the FP32 corrections of that physics
                                 (mech, thermal, moisture) stopped contracting the FP64
                                 residual (less than a half per step over three steps) and
                                 an FP64 block-Jacobi correction solve finished it          */
    int32_t spd;              /* 1: the symmetric parts of C_bar, K_bar, D_bar are positive
                                 definite (Cholesky test)                                     */
    double hill_mandel_gap;   /* largest over C, K, D of ||A_avg - A||_F / ||A||_F, A the
                                 reported (energy-form) matrix and A_avg the plain volume
                                 average of stress / flux (Sec. 2, Eq. macro_stress): the
                                 defect of the Hill-Mandel equality (Eq. Hill_prin), zero
                                 up to rounding for the exact discrete solution           */
} chom_report;

/* Fill *opt with defaults: FP64, two-level preconditioner, max_iter 20000, max_refine 30,
 * rtol 1e-12, inner_rtol 1e-4, c_sat 1.5, no yarn damage, host pointers,
 * null stream.  Always succeeds for non-null opt. */
int chom_default_options(chom_options *opt);

/* Sizes of the n x n x n plain-weave mesh: (n+1)^3 vertices, 6 n^3 tets.
 * Errors: CHOM_EINVAL for n < 1 or n > 1024 or null outputs. */
int chom_mesh_sizes(int32_t n, int32_t *n_vertices, int32_t *n_tets);

/* Generate the synthetic plain-weave RVE on the GPU into caller-allocated
 * device buffers (sizes from chom_mesh_sizes) on the unit cube: the Kuhn
 * lattice above, coordinates i/n, and the yarn tags.  A tet is yarn j if its
 * centroid lies in yarn j's elliptical section (semi-axes 0.2 in-plane, 0.06
 * in z), first hit wins in the order warp y=0.25, warp y=0.75, weft x=0.25,
 * weft x=0.75; warp centrelines z = 0.5 + 0.12 sin(2 pi x + phi), weft
 * z = 0.5 - 0.12 sin(2 pi y + phi), phi = 0, pi.  The fibre axis is the unit
 * centreline tangent at the centroid's abscissa, zero for matrix tets.  The
 * paper models elliptical yarn sections on spline paths (Sec. 1, Table 1);
 * this analytic weave is the synthetic workload geometry.
 * Errors: CHOM_EINVAL (n out of range, null buffer), CHOM_EDEVICE. */
int chom_generate_plain_weave(int32_t n, double *coords, int32_t *tets, int8_t *phase,
                              double *fibre_axis, void *hip_stream);

/* Fibre directions from a potential-flow solve on each yarn (Sec. 6): for yarn
 * j (tets with phase j + 1) Laplace's equation for a potential phi on that
 * yarn's tets alone, phi = 0 on the yarn's vertices on the inlet face lo[d] and
 * phi = 1 on those on the outlet face hi[d] (d = yarn_axis[j], the coordinate
 * the yarn runs along; the paper states no boundary data, this is the reading),
 * no flux through the rest of the yarn's surface; linear elements on the Kuhn
 * lattice (any vertex positions that keep the lattice valid), FP64, Jacobi-
 * preconditioned CG to r.z <= rtol^2 r0.z0 or max_iter steps.  The fibre axis of
 * a yarn tet is its normalised gradient of phi (pointing from inlet to outlet);
 * matrix tets get zero.  The result can be passed as chom_mesh.fibre_axis.
 * mesh: a Kuhn lattice as for chom_rve_create, phase in 0..n_yarns (fibre_axis
 * ignored); fibre_axis [n_tets][3] out, device memory if mesh->on_device, else
 * host.  Work is queued on hip_stream; returns when the output is written.
 * Errors: CHOM_EINVAL (arguments), CHOM_EMESH (not a Kuhn lattice, phase out of
 * range, or a yarn tet with no gradient: a yarn part reaching neither end
 * face), CHOM_ENOCONV (some yarn's solve hit max_iter; directions written),
 * CHOM_EDEVICE, CHOM_ENOMEM. */
int chom_yarn_directions(const chom_mesh *mesh, int32_t n_yarns, const int32_t *yarn_axis, double rtol,
                         int32_t max_iter, double *fibre_axis, void *hip_stream);

/* Create an RVE handle: copies the mesh to the device, checks it (CHOM_EMESH),
 * tabulates the order-p hierarchic basis (order 2, 3 or 4), precomputes
 * element geometry and the constraint rows of bc_type.  opt may be NULL
 * (defaults).  *out receives a caller-owned handle.  Errors: CHOM_EINVAL,
 * CHOM_EMESH, CHOM_EDEVICE, CHOM_ENOMEM. */
int chom_rve_create(const chom_mesh *mesh, const chom_materials *mat, int32_t bc_type,
                    int32_t order, const chom_options *opt, chom_rve **out);

/* Matrix damage under time-varying exposure at n macro Gauss points (Sec. 4,
 * Eq. Eq_Model_RateForm): d(1 - omega)/dt = -gamma(c) alpha(T) (1 - omega) with
 * alpha, gamma as in chom_params, stepped with implicit (backward) Euler as the
 * paper states: over step k, (1 - omega)_k = (1 - omega)_{k-1} /
 * (1 + gamma(c_k) alpha(T_k) dt_k).  For constant exposure it tends to the
 * closed form of chom_params (Eq. Eq_Model_final1) at first order in dt.
 * Inputs: T_celsius [m][n] and c_wt [m][n] (step-major: step k of every point
 * is row k), dt_years [m], keep0 [n] (nullable: 1, undamaged), factors [n][8]
 * (nullable: 1; copied into params_out).  Outputs (at least one non-null):
 * keep [m][n], (1 - omega) after every step; params_out [n], for each point an
 * equivalent constant-exposure record -- T = 60 C, c = c_sat (gamma = 1) and the
 * exposure time after which the closed form gives the final (1 - omega) -- that
 * chom_homogenise, chom_batch_homogenise and the surrogate take as they are
 * (use the same c_sat there).  device_ptrs: 1 if every array is device memory,
 * 0 if every array is host memory.  Work is queued on hip_stream (NULL: null
 * stream); the call returns when the outputs are written.
 * Errors: CHOM_EINVAL (sizes, null arrays, c_sat <= 0, or an exposure outside the
 * law's domain: T >= T_g, c < 0, dt < 0, keep0 outside (0, 1]), CHOM_EDEVICE,
 * CHOM_ENOMEM. */
int chom_damage_history(int64_t n, int32_t m, const double *T_celsius, const double *c_wt, const double *dt_years,
                        const double *keep0, const double *factors, double c_sat, int32_t device_ptrs,
                        void *hip_stream, double *keep, chom_params *params_out);

/* Fully nested multi-scale run (FE^2, paper Sec. 3 and Sec. 5): a synthetic
 * macro box [0, lx] x [0, ly] x [0, lz] on an nx x ny x nz Kuhn lattice of
 * linear (P1) tets, one Gauss point (its centroid) per tet.  Per time step:
 *  - macro heat and moisture transport (Eq. Eq_field, discretised as in
 *    Eq. Eq_field_disc: capacity (consistent P1 mass) and conductivity
 *    matrices, implicit Euler in time): heat_capacity * dT/dt = div(K_T grad T),
 *    dc/dt = div(D_c grad c), with K_T, D_c the RVE's homogenised conductivity
 *    and diffusivity of the undegraded record (homogenised once: they do not
 *    depend on the damage), T = T_top and c = c_top on the face z = lz, no flux
 *    elsewhere, T = T0 and c = c0 at t = 0; time in years, lengths in the units
 *    the homogenised coefficients are taken in (a synthetic setting: the paper's
 *    macro geometry and loads are not specified);
 *  - at every Gauss point the damage of the matrix by the rate form of Sec. 4
 *    (Eq. Eq_Model_RateForm), implicit Euler with the step's end values of T
 *    and c (the mean of the tet's vertex values), as chom_damage_history with
 *    the RVE's c_sat;
 *  - at every Gauss point the mechanical RVE solve with that damage (the RVE
 *    handle `rve`, one batched chom_homogenise call per step) giving C_bar;
 *  - macro linear elasticity with these C_bar: u_x = 0 on x = 0, u_x =
 *    strain_x * lx on x = lx, u_y = 0 on y = 0, u_z = 0 on z = 0, other faces
 *    free; out->reaction[step] is the x-force on the face x = lx.
 * Macro systems: FP64, Jacobi-preconditioned CG (one workgroup per system) to
 * r.z <= macro_rtol^2 r0.z0.  factors [8] (nullable: all 1) scale the RVE's
 * properties at every Gauss point (as in chom_params).  Outputs (host memory,
 * each nullable): T, c [steps + 1][nv] vertex fields (nv = (nx+1)(ny+1)(nz+1),
 * x fastest), keep [steps][ngp] (ngp = 6 nx ny nz, tet order of
 * chom_generate_plain_weave's lattice), reaction [steps], u [nv][3] and
 * C_bar [ngp][21] of the last step.  The RVE's own options (precision,
 * tolerances, host or device pointers) apply to its solves.  With `surrogate`
 * set (a trained ensemble with the RVE's c_sat and at least two members), the
 * Gauss points' C_bar come from chom_homogenise_surrogate with this RVE as the
 * fallback for records whose disagreement exceeds surrogate_thresh (the
 * transport coefficients still come from one RVE solve); out->n_fallback
 * counts the fallback solves over all steps.
 * Errors: CHOM_EINVAL (arguments; also T0 or T_top at or above the law's glass
 * transition T_g = 126 C, negative c0 or c_top, or a Gauss-point exposure that
 * leaves the law's domain), CHOM_ENOCONV (a macro solve or an RVE solve did not
 * converge; outputs written), CHOM_EMATERIAL, CHOM_EDEVICE, CHOM_ENOMEM. */
typedef struct {
    int32_t nx, ny, nz;          /* macro cells along x, y, z (>= 1)                          */
    double lx, ly, lz;           /* box edge lengths (> 0)                                      */
    double heat_capacity;        /* rho c_p (> 0)                                               */
    double T0, c0;               /* initial temperature (Celsius) and moisture (wt%)            */
    double T_top, c_top;         /* exposure on z = lz                                          */
    double dt_years;             /* time step (> 0)                                             */
    int32_t steps;               /* time steps (>= 1)                                           */
    double strain_x;             /* macro stretch of the uniaxial test                          */
    double macro_rtol;           /* macro CG tolerance (e.g. 1e-10)                             */
    int32_t macro_max_iter;      /* macro CG step cap                                           */
    const double *factors;       /* [8] or NULL                                                 */
    chom_mlp *surrogate;         /* NULL: an RVE solve at every Gauss point                     */
    double surrogate_thresh;     /* fallback threshold on the ensemble disagreement             */
} chom_fe2_problem;

typedef struct {
    double *T, *c;               /* [steps + 1][nv]                                             */
    double *keep;                /* [steps][ngp]                                                */
    double *reaction;            /* [steps]                                                     */
    double *u;                   /* [nv][3], last step                                          */
    double *C_bar;               /* [ngp][21], last step                                        */
    int32_t macro_iters[3];      /* largest CG step count of the heat, moisture, mechanics solves */
    int64_t n_fallback;          /* RVE fallback solves of the surrogate, all steps             */
} chom_fe2_output;

int chom_fe2_run(chom_rve *rve, const chom_fe2_problem *prob, chom_fe2_output *out);

/* Homogenise the RVE for `batch` parameter records: 6 mechanical + 3 thermal
 * + 3 moisture load cases each.  Outputs: C_hom [batch][21], K_hom [batch][6],
 * D_hom [batch][6], rep [batch] (rep may be NULL; rep is always host memory).
 * Returns CHOM_ENOCONV (results written, rep.status set) if a load case hit the
 * iteration cap, CHOM_EMATERIAL if a record gives a non-positive-definite
 * material, CHOM_EINVAL / CHOM_EDEVICE / CHOM_ENOMEM otherwise (CHOM_EINVAL
 * also for an RVE whose operator tile boxes exceed 2^31 values for one problem,
 * far beyond device memory for any supported order). */
int chom_homogenise(chom_rve *rve, const chom_params *params, int32_t batch,
                    double *C_hom, double *K_hom, double *D_hom, chom_report *rep);

/* Time the matrix-free operator kernel that chom_homogenise launches for
 * `physics` (0: mechanical, 6 load cases; 1: thermal + moisture, 3 load cases
 * each) at the handle's precision (FP32 operator when CHOM_FP32_REFINED):
 * `reps` back-to-back launches with the same grid and problem table as the last
 * chom_homogenise call, on the handle's stream, between two HIP events; the
 * operands are that call's workspace vectors (their contents are overwritten).
 * Outputs: average milliseconds per launch, tets processed per launch (tets x
 * problems) and problems per launch (either pointer may be NULL).
 * Errors: CHOM_EINVAL (no prior chom_homogenise, bad argument), CHOM_EDEVICE. */
int chom_time_operator(chom_rve *rve, int32_t physics, int32_t reps, double *ms_per_launch,
                       int64_t *tets_per_launch, int32_t *problems_per_launch);

/* Release a handle (NULL is ignored).  Batches that list the handle must be
 * destroyed first. */
void chom_rve_destroy(chom_rve *rve);

/* ---------------------------------------------------------------- general tet meshes
 * RVEs on any conforming tet mesh of the box [lo, hi] (the paper's RVE is an
 * unstructured mesh of its spline yarn geometry, Sec. 1, Table 1; the lattice
 * handles above need the Kuhn lattice).  Order-2 hierarchic elements on the
 * mesh's vertices and edges (numbered by the library), the element operator
 * of the lattice path applied one thread per tet with FP64 atomic assembly,
 * point-block Jacobi PCG in FP64 per load case with the energy-relative
 * stopping test of chom_options.rtol (Sec. 2, Eqs. eq_RVE_disc_Eqs,
 * Eq_C_stress, eq_homo_flux: the same 6 + 3 + 3 load cases and energy-form
 * averages as chom_homogenise).
 * bc: CHOM_BC_DIRICHLET (linear displacement / temperature / concentration on
 * every boundary vertex and boundary edge) or CHOM_BC_PERIODIC (the faces
 * x_d = hi_d must match x_d = lo_d vertex for vertex and edge for edge; the
 * class of the corner lo is pinned, which fixes the translations and leaves
 * C_bar unchanged) or CHOM_BC_NEUMANN (uniform traction, Sec. 2 item 3: the
 * fluctuation is held to zero surface moments int u_i n_j dS and zero mean
 * int u_i dV, and PCG runs on that subspace with the projection
 * z = M^-1 (r - C^T y), y = (C M^-1 C^T)^-1 C M^-1 r).
 * opt: precision must be CHOM_FP64 (precond is ignored: point-block Jacobi);
 * rtol, max_iter, c_sat, degrade_yarn, device_ptrs (params and outputs of
 * chom_urve_homogenise) and hip_stream are used.  The mesh arrays are copied.
 * Errors: CHOM_EINVAL (arguments, options), CHOM_EMESH (vertex outside the box,
 * vertex id out of range, degenerate tet, tets not filling the box, phase out
 * of 0..4, non-unit yarn axis, periodic faces that do not match, no vertex at
 * the corner lo), CHOM_EMATERIAL, CHOM_EDEVICE, CHOM_ENOMEM. */
typedef struct chom_urve chom_urve;
int chom_urve_create(const chom_mesh *mesh, const chom_materials *mat, int32_t bc, const chom_options *opt,
                     chom_urve **out);

/* P2 nodes (vertices + edges) and free unknowns (per component) of a handle. */
int chom_urve_sizes(const chom_urve *u, int64_t *n_nodes, int64_t *n_unknowns);

/* Homogenise `batch` parameter records (in chunks of up to 16 whose load cases
 * share every launch; fewer on very large meshes): outputs and report
 * as for chom_homogenise (refine_steps and fp64_fallback are 0; the
 * Hill-Mandel gap compares the energy form with the volume average of stress
 * and flux).  Errors: CHOM_ENOCONV (results written), CHOM_EINVAL (records
 * outside the degradation law), CHOM_EDEVICE, CHOM_ENOMEM. */
int chom_urve_homogenise(chom_urve *u, const chom_params *params, int32_t batch, double *C_hom, double *K_hom,
                         double *D_hom, chom_report *rep);

/* Release a general-mesh handle (NULL is ignored). */
void chom_urve_destroy(chom_urve *u);

/* Yarn tags of any tet mesh of the unit cube by the synthetic weave of
 * chom_generate_plain_weave (the same centroid test and tangent): phase [n_tets]
 * and fibre_axis [n_tets][3] out; coords [n_vertices][3], tets [n_tets][4] in.
 * device_ptrs: 1 if all four arrays are device memory.  Runs on the GPU.
 * Errors: CHOM_EINVAL, CHOM_EMESH (vertex id out of range), CHOM_EDEVICE. */
int chom_tag_plain_weave(const double *coords, int64_t n_vertices, const int32_t *tets, int64_t n_tets,
                         int32_t device_ptrs, int8_t *phase, double *fibre_axis);

/* ---------------------------------------------------------------- batches
 * One macro Gauss point per item (the FE^2 setting of Sec. 5, where every macro
 * Gauss point carries its own RVE): item i is homogenised on RVE rves[i] with
 * parameter record params[i].  Handles may repeat (items sharing a mesh) and may
 * differ in size and boundary condition; all items and all 12 load cases run in
 * the same kernel launches (one problem table per physics), the CG iterations
 * replayed from a captured HIP graph, with device-side convergence flags so
 * finished items cost only an early exit.  opt may be NULL (the first handle's
 * options).  The handles must outlive the batch.
 * Errors: CHOM_EINVAL, CHOM_EDEVICE, CHOM_ENOMEM. */
int chom_batch_create(chom_rve *const *rves, int32_t n, const chom_options *opt, chom_batch **out);

/* Homogenise every item of the batch: params [n], C_hom [n][21], K_hom [n][6],
 * D_hom [n][6], rep [n] (nullable, host).  Same conventions and errors as
 * chom_homogenise.  If the environment variable CHOM_AUTOTUNE is set, the first
 * call times the operator's load-case grouping (1, 2 or 3 load cases per
 * workgroup) and the vector kernels' grid (128..1024 workgroups per item) on
 * this batch and keeps the fastest; results are cached per device, precision
 * and size mix (and persisted to the file named by CHOM_TUNE_FILE if set). */
int chom_batch_homogenise(chom_batch *batch, const chom_params *params, double *C_hom, double *K_hom,
                          double *D_hom, chom_report *rep);

/* Launch shape in use: load cases per operator workgroup and vector
 * workgroups per item, for the mechanical and scalar classes (any pointer may
 * be NULL).  Errors: CHOM_EINVAL. */
int chom_batch_launch_config(const chom_batch *batch, int32_t *rg_mech, int32_t *rg_scal, int32_t *nwg_mech,
                             int32_t *nwg_scal);

/* As chom_time_operator, for a batch. */
int chom_batch_time_operator(chom_batch *batch, int32_t physics, int32_t reps, double *ms_per_launch,
                             int64_t *tets_per_launch, int32_t *problems_per_launch);

/* Release a batch (NULL is ignored). */
void chom_batch_destroy(chom_batch *batch);

/* ---------------------------------------------------------------- learned surrogate
 * An ensemble of small networks that maps a parameter record (temperature,
 * moisture, exposure time, eight property factors) to the homogenised
 * C_bar, K_bar, D_bar of one RVE, trained on that RVE's own solves, with the RVE
 * solve as fallback where the ensemble disagrees.  The surrogate is not part of
 * the paper; it reads the record through the paper's degradation law (Sec. 4,
 * Eq. Eq_Model_final1): its ten features are log(1 - omega), (1 - omega) and
 * the eight factors.
 *
 * Network of each member: 10 -> 256 -> 256 -> 256 -> 36, GELU (z Phi(z)) on the
 * hidden layers.  The 36 outputs encode the 21 + 6 + 6 entries of
 * chom_homogenise per block (C, K, D) as the log of the block's Frobenius norm
 * followed by the block divided by that norm; decoding rescales the predicted
 * direction to unit norm, so the error of a block is relative to its size.
 * Features and encoded outputs are standardised with per-column mean and
 * population deviation of the training set.  Weights and activations enter the products as
 * bfloat16 (round to nearest even) with FP32 accumulation; biases, the loss,
 * gradients and Adam moments are FP32; standardisation is FP64.
 *
 * Flat parameter layout of one member (FP32, row-major [out][in]):
 *   W1 [256][10], b1 [256], W2 [256][256], b2 [256], W3 [256][256], b3 [256],
 *   W4 [36][256], b4 [36]                       (143,652 numbers)
 * Standardisation record (FP64, 92 numbers): feature means [10], feature
 * deviations [10], encoded-output means [36], encoded-output deviations [36].
 *
 * Disagreement of a point: the largest over the C, K, D blocks of
 * ||s||_F / ||m||_F, with m the member mean and s the sample standard deviation
 * over members, both in physical units, and ||.||_F the Frobenius norm of the
 * full symmetric matrix (off-diagonal entries counted twice).
 *
 * Pointer convention: params [n] (chom_params), C [n][21], K [n][6], D [n][6],
 * disagreement [n] and used_fallback [n] are device pointers when
 * chom_mlp_options.device_ptrs is set, else host pointers.  Weight and
 * standardisation arrays are always host pointers. */

typedef struct {
    int32_t members;        /* ensemble size, 1..8 (default 5)                           */
    int32_t device_ptrs;    /* 1: bulk arrays are device pointers                         */
    uint64_t seed;          /* initial weights (U(-a, a), a = sqrt(3 / fan_in), zero biases) and shuffles */
    double c_sat;           /* moisture of full saturation in the degradation law (wt%), default 1.5 */
    void *hip_stream;       /* hipStream_t or NULL (the library's own stream)           */
} chom_mlp_options;

typedef struct {
    int32_t epochs;         /* passes over the training set (default 300)                 */
    int32_t batch;          /* minibatch rows, 1..256 (default 256)                       */
    float lr, lr_final;     /* Adam step size, cosine-decayed from lr to lr_final over the call (2e-3, 2e-5) */
    float beta1, beta2, eps;/* Adam constants (0.9, 0.999, 1e-8)                          */
    int32_t refit_normalisation; /* 1: standardise with this training set's statistics (default 1) */
} chom_mlp_train_options;

int chom_mlp_default_options(chom_mlp_options *opt);
int chom_mlp_default_train_options(chom_mlp_train_options *opt);

/* Create an ensemble with seeded initial weights.  opt may be NULL (defaults).
 * Errors: CHOM_EINVAL, CHOM_EDEVICE, CHOM_ENOMEM. */
int chom_mlp_create(const chom_mlp_options *opt, chom_mlp **out);

/* Parameters per member (143,652) and members.  Errors: CHOM_EINVAL. */
int chom_mlp_sizes(const chom_mlp *mlp, int64_t *params_per_member, int32_t *members);

/* Replace (set) or read (get) one member's FP32 master weights, flat layout
 * above, host memory.  Setting also clears that member's Adam moments and, for
 * every member, the Adam step count.  Errors: CHOM_EINVAL, CHOM_EDEVICE. */
int chom_mlp_set_weights(chom_mlp *mlp, int32_t member, const float *flat);
int chom_mlp_get_weights(const chom_mlp *mlp, int32_t member, float *flat);

/* Replace or read the standardisation record (92 doubles, host).  Deviations
 * must be positive.  Errors: CHOM_EINVAL (and for get: no record yet). */
int chom_mlp_set_normalisation(chom_mlp *mlp, const double *record);
int chom_mlp_get_normalisation(const chom_mlp *mlp, double *record);

/* Train every member on n (record, result) pairs: minibatch Adam on the mean
 * squared error of the standardised outputs (each member shuffles the set
 * independently every epoch; all members advance together, every minibatch
 * step a fixed sequence of kernels replayed from HIP graphs; the call returns
 * when training has finished).  loss_history
 * [members][epochs] (host, nullable) receives each epoch's mean loss.  Calls
 * may be repeated (training continues).  1 <= n < 2^31.
 * Errors: CHOM_EINVAL (records outside the degradation law's domain, sizes),
 * CHOM_EDEVICE, CHOM_ENOMEM. */
int chom_mlp_train(chom_mlp *mlp, const chom_params *params, const double *C, const double *K, const double *D,
                   int64_t n, const chom_mlp_train_options *opt, float *loss_history);

/* Loss of one member on n pairs and its gradient with respect to the flat
 * parameters (grad [143,652], host), without updating anything; the forward
 * and backward kernels of chom_mlp_train, for checking.  Needs a
 * standardisation record.  Errors: CHOM_EINVAL, CHOM_EDEVICE, CHOM_ENOMEM. */
int chom_mlp_loss_grad(chom_mlp *mlp, int32_t member, const chom_params *params, const double *C,
                       const double *K, const double *D, int64_t n, double *loss, float *grad);

/* chom_mlp_loss_grad without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving or training loops,
 * harnesses that forbid hipMalloc).  The same kernels and results as
 * chom_mlp_loss_grad, but every pointer is a device pointer -- params [n]
 * (chom_params), C [n][21], K [n][6], D [n][6] in, *loss (one double) and grad
 * [143,652] (FP32) out -- whatever the handle's device_ptrs setting, and the
 * working memory (standardised rows, flag, training scratch; about 2.7 MB) is a
 * static array of the library that each device holds until the process ends.
 * n is limited to 4096 records (CHOM_EINVAL beyond).  Calls that overlap on one
 * device share that array and race: serialise them.  Work is queued on the
 * handle's stream; the call returns after the input check has been read back.
 * Errors: CHOM_EINVAL (argument, n, member, no standardisation record, records
 * outside the degradation law's domain), CHOM_EDEVICE. */
int chom_mlp_loss_grad_noalloc(chom_mlp *mlp, int32_t member, const chom_params *params, const double *C,
                               const double *K, const double *D, int64_t n, double *loss, float *grad);

/* Ensemble prediction for n records: member mean in physical units (C, K, D)
 * and the disagreement (nullable).  Needs a standardisation record.
 * Errors: CHOM_EINVAL (records outside the law's domain), CHOM_EDEVICE. */
int chom_mlp_predict(chom_mlp *mlp, const chom_params *params, int64_t n, double *C, double *K, double *D,
                     double *disagreement);

/* Surrogate with fallback: predict all n records, then re-solve with the RVE
 * (chom_homogenise on `fallback`, in chunks of at most `chunk` records; 0 means
 * 256) every record whose disagreement exceeds thresh, overwriting its
 * prediction.  used_fallback [n] (uint8, nullable) flags the re-solved records;
 * *n_fallback (nullable, host) receives their count.  The RVE must use the same
 * c_sat as the ensemble.  Needs members >= 2.
 * Errors: those of chom_mlp_predict and chom_homogenise (CHOM_ENOCONV: results
 * written, some fallback solve did not converge). */
int chom_homogenise_surrogate(chom_mlp *mlp, chom_rve *fallback, const chom_params *params, int64_t n,
                              double thresh, int32_t chunk, double *C, double *K, double *D,
                              double *disagreement, uint8_t *used_fallback, int64_t *n_fallback);

/* Release an ensemble (NULL is ignored). */
void chom_mlp_destroy(chom_mlp *mlp);

/* Message of the last failing call on this thread ("" if none). */
const char *chom_last_error(void);

/* ---------------------------------------------------------------- host-only helpers
 * These run on the CPU and need no GPU; they expose the library's own host
 * arithmetic for inspection. */

/* Material constants of one record as used by the kernels.  out_mech[10]:
 * per phase (matrix, yarn) the five transversely isotropic invariants
 * (lambda, mu_T, alpha, mu_L - mu_T, beta) of
 *   sigma = lambda tr(e) I + 2 mu_T e + alpha ((a.e.a) I + tr(e) A)
 *         + 2 (mu_L - mu_T)(A e + e A) + beta (a.e.a) A,   A = a a^T;
 * out_therm[4], out_moist[4]: per phase (k_T, k_L - k_T) of k_T I + (k_L - k_T) A;
 * *omega_keep: the matrix damage factor.  params may be NULL (no factors, no
 * damage).  Errors: CHOM_EINVAL, CHOM_EMATERIAL. */
int chom_material_constants(const chom_materials *mat, const chom_params *params, double c_sat,
                            int32_t degrade_yarn, double *out_mech, double *out_therm,
                            double *out_moist, double *omega_keep);

/* One element of the order-2 operator evaluated on the host with the same code
 * the kernels run: y = K_e u for a tet with barycentric-coordinate gradients
 * grad_lam [4][3], volume vol, fibre axis [3] and the five invariants inv5 of
 * chom_material_constants (ncomp = 3; for ncomp = 1 inv5[0..1] = (k_T, k_L - k_T)).
 * u, y: [10][ncomp], DOFs ordered vertices 0..3 then edges (01, 02, 03, 12,
 * 13, 23); vertex functions lam_a, edge functions 4 lam_a lam_b.
 * Errors: CHOM_EINVAL. */
int chom_element_apply_host(int32_t ncomp, const double *grad_lam, double vol, const double *axis,
                            const double *inv5, const double *u, double *y);

/* Tables of the order-p hierarchic basis (p = 3 or 4) that the order-p kernels
 * use, for inspection: *n_e local functions (20 or 35) and *m = dim P_{p-1};
 * S [9][n_e][n_e] = (1/|e|) int d_k phi_i d_l phi_j (k, l over the reference
 * coordinates xi_1..3 = lam_1..3, entry (k*3 + l)), as the kernels form it from
 * their derivative tables; W [n_e] = (1/|e|) int phi_i; Wd [3][n_e] =
 * (1/|e|) int d phi_i / d xi_k; offsets [6][n_e][3] = lattice point of each local
 * DOF per Kuhn tet type, in units of 1/p cell from the cell origin.  Local order:
 * vertices, edges (01, 02, 03, 12, 13, 23; p-1 each), faces (omitting vertex
 * 0, 1, 2, 3; (p-1)(p-2)/2 each), interior.  Functions: see hp_tables.cpp of the
 * library sources (paper Sec. 1, Sec. 7 name only the hierarchic family).  Any
 * output pointer may be NULL.  Errors: CHOM_EINVAL (order). */
int chom_basis_tables_host(int32_t order, int32_t *n_e, int32_t *m, double *S, double *W, double *Wd,
                           int32_t *offsets);

/* Values of the order-p basis functions (p = 3, 4) at barycentric point lam [4]
 * (out [n_e]).  Errors: CHOM_EINVAL. */
int chom_basis_eval_host(int32_t order, const double *lam, double *out);

/* Library version string. */
const char *chom_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CHOM_H */
