// C ABI of libchom: argument checking, mesh validation, material constants,
// batches and workspaces, the host side of the solver (PCG loop captured in a
// HIP graph, refinement loop) and the launch autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

#include "hp.h"
#include "internal.h"

namespace chom {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

// ------------------------------------------------------------------ materials
static const double kBeta = -0.001682;     // per day (Sec. 4, Eq. Eq_alphaT_LSF)
static const double kTgC = 126.0;          // glass transition (Sec. 4)
static const double kKelvin = 273.15;
static const double kDaysPerYear = 365.25;

// Degradation factor (1 - omega) = exp(-gamma(c) alpha(T) t), Eq. Eq_Model_final1.
static bool damage_factor(const chom_params *pr, double c_sat, double *keep) {
    if (!pr) { *keep = 1.0; return true; }
    const double TK = pr->T_celsius + kKelvin, TgK = kTgC + kKelvin;
    const double arg = 1.0 - TK / TgK;
    if (!(arg > 0.0) || !(c_sat > 0.0) || !(pr->c_wt >= 0.0) || !(pr->t_years >= 0.0)) return false;
    const double alpha = kBeta * std::log(arg);
    const double gamma = pr->c_wt / c_sat;
    *keep = std::exp(-gamma * alpha * pr->t_years * kDaysPerYear);
    return std::isfinite(*keep) && *keep > 0.0;
}

// Local transversely isotropic stiffness (fibre along e1) -> the five invariants.
static bool transiso_invariants(double E1, double E2, double G12, double nu12, double nu23, double out[5]) {
    if (!(E1 > 0 && E2 > 0 && G12 > 0)) return false;
    const double s11 = 1.0 / E1, s22 = 1.0 / E2, s12 = -nu12 / E1, s23 = -nu23 / E2;
    const double S[3][3] = {{s11, s12, s12}, {s12, s22, s23}, {s12, s23, s22}};
    const double det = S[0][0] * (S[1][1] * S[2][2] - S[1][2] * S[2][1]) -
                       S[0][1] * (S[1][0] * S[2][2] - S[1][2] * S[2][0]) +
                       S[0][2] * (S[1][0] * S[2][1] - S[1][1] * S[2][0]);
    const double m2 = S[0][0] * S[1][1] - S[0][1] * S[1][0];
    if (!(S[0][0] > 0 && m2 > 0 && det > 0)) return false;
    const double C11 = (S[1][1] * S[2][2] - S[1][2] * S[2][1]) / det;
    const double C12 = -(S[1][0] * S[2][2] - S[1][2] * S[2][0]) / det;
    const double C22 = (S[0][0] * S[2][2] - S[0][2] * S[2][0]) / det;
    const double C23 = -(S[0][0] * S[2][1] - S[0][1] * S[2][0]) / det;
    const double lam = C23;
    const double muT = 0.5 * (C22 - C23);
    const double alpha = C12 - lam;
    const double muL = G12;
    const double beta = C11 - lam - 2.0 * muT - 2.0 * alpha - 4.0 * (muL - muT);
    if (!(muT > 0)) return false;
    out[0] = lam;
    out[1] = muT;
    out[2] = alpha;
    out[3] = muL - muT;
    out[4] = beta;
    return true;
}

static int material_constants(const chom_materials *m, const chom_params *pr, double c_sat, int degrade_yarn,
                              double mech[10], double therm[4], double moist[4], double *keep_out) {
    double f[8] = {1, 1, 1, 1, 1, 1, 1, 1};
    if (pr)
        for (int i = 0; i < 8; ++i) f[i] = pr->factor[i];
    for (int i = 0; i < 8; ++i)
        if (!(f[i] > 0) || !std::isfinite(f[i])) {
            set_error("property factors must be positive and finite");
            return CHOM_EMATERIAL;
        }
    double keep;
    if (!damage_factor(pr, c_sat, &keep)) {
        set_error("exposure parameters outside the degradation law's domain (T < T_g, c, t >= 0)");
        return CHOM_EMATERIAL;
    }
    const double E = m->E * f[0] * keep, nu = m->nu * f[1];
    if (!(E > 0) || !(nu > -1.0 && nu < 0.5)) {
        set_error("matrix stiffness not positive definite");
        return CHOM_EMATERIAL;
    }
    const double lam = E * nu / ((1 + nu) * (1 - 2 * nu)), mu = E / (2 * (1 + nu));
    mech[0] = lam; mech[1] = mu; mech[2] = 0; mech[3] = 0; mech[4] = 0;
    const double ys = degrade_yarn ? keep : 1.0;
    if (!transiso_invariants(m->E1 * f[4] * ys, m->E2 * f[4] * ys, m->G12 * f[4] * ys, m->nu12 * f[5],
                             m->nu23 * f[5], mech + 5)) {
        set_error("yarn stiffness not positive definite");
        return CHOM_EMATERIAL;
    }
    const double km = m->k * f[2], Dm = m->D * f[3];
    const double k1 = m->k1 * f[6], k2 = m->k2 * f[6], D1 = m->D1 * f[7], D2 = m->D2 * f[7];
    if (!(km > 0 && Dm > 0 && k1 > 0 && k2 > 0 && D1 > 0 && D2 > 0)) {
        set_error("conductivity/diffusivity not positive");
        return CHOM_EMATERIAL;
    }
    therm[0] = km; therm[1] = 0; therm[2] = k2; therm[3] = k1 - k2;
    moist[0] = Dm; moist[1] = 0; moist[2] = D2; moist[3] = D1 - D2;
    if (keep_out) *keep_out = keep;
    return CHOM_OK;
}

// ------------------------------------------------------------------ workspaces
// A captured run of CG iterations (the kernel sequence is fixed by the buffers).
struct GraphCache {
    hipGraphExec_t exec = nullptr;
    const void *key = nullptr;   // buffer identity the graph was captured for
    int iters = 0;
    unsigned long long gen = 0;  // workspace generation it was captured for
    const void *probs = nullptr; // problem range it was captured for
    int nprob = 0;
    ~GraphCache() { reset(); }
    void reset() {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
        key = nullptr;
        iters = 0;
        gen = 0;
        probs = nullptr;
        nprob = 0;
    }
};

template <int C, int R> struct ClassWS {
    static constexpr int MS = (C == 3) ? 6 : 1;
    Launch L{};
    hipStream_t stream = nullptr;        // the class's stream (mechanics: the batch stream)
    hipStream_t stream_b = nullptr;      // the second CG chain's stream
    long long total_vals = 0, total_pts = 0, total_q = 0;
    int nwg_gram = 0, nwg_avg = 0;
    unsigned long long gen = 0;          // bumped whenever the launch shape may change
    DevBuf<Prob> probs;
    DevBuf<double> b, x64, r64, q64;
    DevBuf<double> xd, rd, pd, qd;
    DevBuf<float> xf, rf, pf, qf, r32;
    DevBuf<double> diag, minv64, ginv64, ginv32, ycoef;
    DevBuf<float> minv32;
    DevBuf<ColState> cols, cols_outer;
    DevBuf<int> active, active_outer, bad;
    DevBuf<double> partial, avg_out;
    DevBuf<double> acc, accpq;           // striped CG accumulators (see ACC_STRIPES)
    DevBuf<double> ef64;                 // orders 3, 4: element factors
    DevBuf<float> ef32;
    // two-level preconditioner: FP64 setup arrays, the solve-precision copies,
    // level vectors, W = V P^T C^T, Gram matrices (non-inverted) and C B C^T inverse
    DevBuf<double> mgA64, mgD64, mgrows1, gmat, ginv_mg;
    DevBuf<float> mgA32, mgD32, mgr32, mgxp32, mgres32, mgx32, mgW32;
    DevBuf<double> mgr64, mgxp64, mgres64, mgx64, mgW64;
    DevBuf<double> avg_corr;             // Hill-Mandel gap terms (1/V) u_i . r_j [prob][NC][R]
    DevBuf<ColState> cols_tmp, cols_fb;  // final-residual projection; mask of the FP64 fallback solve
    DevBuf<ColState> cols_flush;         // CG chain compaction: pending updates of the leaving problems
    DevBuf<int> active_tmp;
    std::vector<ColState> h_cols, h_cols_outer, h_cols_tmp;
    HostBuf<int> h_poll;               // pinned: per-problem active flags polled between graph chunks
    std::vector<int> refine_steps;
    std::vector<int> fallback;         // per problem: an FP64 solve finished a stalled refinement
    GraphCache graph64, graph32, graph64b, graph32b;   // per precision and CG chain
};

}  // namespace chom

using namespace chom;

struct chom_rve {
    int n = 0, bc = 0, order = 2;
    double lo[3], hi[3];
    chom_materials mat;
    chom_options opt;
    Geo geo;
    DevBuf<double4> elem64;
    DevBuf<float4> elem32;
    DevBuf<double> geo64;
    DevBuf<float> geo32;
    DevBuf<double> rows;
    DevBuf<int> hoff;                                    // orders 3, 4: basis tables
    DevBuf<double> hW, hWd, hSd, hDA64, hDB64;
    DevBuf<int> mg_nbr, mg_child, mg_par;               // coarse-level index tables
    DevBuf<float> hDA32, hDB32;
    std::unique_ptr<chom_batch> self;   // batch of this RVE alone (chom_homogenise)
    int self_size = 0;
    ~chom_rve();
};

struct chom_batch {
    std::vector<chom_rve *> entries;    // one per batch item (handles may repeat)
    std::vector<chom_rve *> distinct;   // distinct handles, index = Prob.geo
    std::vector<int> geo_of;            // entry -> index in distinct
    chom_options opt;
    hipStream_t stream = nullptr;
    hipStream_t stream2 = nullptr;      // scalar class, run concurrently with the mechanical one
    bool own_stream = false;
    DevBuf<Geo> geos;
    ClassWS<3, 6> mech;
    ClassWS<1, 3> scal;
    int rg_mech = 2, rg_scal = 3;       // load cases per operator workgroup
    int nwg_mech = 0, nwg_scal = 0;     // vector workgroups per problem (0: default)
    bool tuned = false;
    ~chom_batch() {
        for (GraphCache *g : {&mech.graph64, &mech.graph32, &mech.graph64b, &mech.graph32b, &scal.graph64,
                              &scal.graph32, &scal.graph64b, &scal.graph32b})
            g->reset();
        if (own_stream && stream) (void)hipStreamDestroy(stream);
        if (stream2) (void)hipStreamDestroy(stream2);
        if (mech.stream_b) (void)hipStreamDestroy(mech.stream_b);
        if (scal.stream_b) (void)hipStreamDestroy(scal.stream_b);
    }
};

chom_rve::~chom_rve() { self.reset(); }

namespace chom {

// ------------------------------------------------------------------ autotune cache
// Process-wide cache of tuned launch shapes, keyed by device, physics,
// precision and problem sizes; optionally persisted to $CHOM_TUNE_FILE.
static std::mutex g_tune_mu;
static std::map<std::string, std::pair<int, int>> g_tune;
static bool g_tune_loaded = false;

static void tune_load() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("CHOM_TUNE_FILE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char key[512];
    int a, b;
    while (std::fscanf(f, "%511s %d %d", key, &a, &b) == 3) g_tune[key] = {a, b};
    std::fclose(f);
}

static void tune_store(const std::string &key, int a, int b) {
    g_tune[key] = {a, b};
    const char *path = std::getenv("CHOM_TUNE_FILE");
    if (!path) return;
    FILE *f = std::fopen(path, "w");
    if (!f) return;
    for (auto &kv : g_tune) std::fprintf(f, "%s %d %d\n", kv.first.c_str(), kv.second.first, kv.second.second);
    std::fclose(f);
}

// ------------------------------------------------------------------ class setup
template <int C, int R>
static int setup_class(chom_batch *B, ClassWS<C, R> &W, std::vector<Prob> &hp, int rg, int nwg_override) {
    constexpr int MS = ClassWS<C, R>::MS;
    const int nprob = (int)hp.size();
    long long voff = 0, doff = 0, qoff = 0, eoff = 0, moff = 0, max_pts = 0, max_tets = 0;
    constexpr int NQ = (3 * C) * (3 * C + 1) / 2;
    int max_tiles = 0, nr = 0, mg_nlev = 0;
    long long mg_max_pts[MG_MAXLEV] = {}, mg_coarse_pts = 0, mg_deep_pts = 0;
    const bool want_mg = B->opt.precond == CHOM_PRECOND_TWO_LEVEL;
    for (auto &P : hp) {
        const Geo &G = B->distinct[P.geo]->geo;
        // the vector kernels index one problem's tile boxes with 32-bit offsets
        if ((long long)G.ntiles * G.boxpts * R * C > 0x7fffffffLL) {
            set_error("RVE too large: one problem's operator tile boxes exceed 2^31 values");
            return CHOM_EINVAL;
        }
        P.voff = voff;
        P.doff = doff;
        P.qoff = qoff;
        P.eoff = eoff;
        P.moff = moff;
        if (want_mg && G.mg_nlev >= 2) {
            moff += G.mg_pts;
            mg_nlev = std::max(mg_nlev, G.mg_nlev);
            long long deep = 0;
            for (int l = 0; l < G.mg_nlev; ++l) {
                const long long np = (long long)G.mg_lw[l] * G.mg_lw[l] * G.mg_lw[l];
                mg_max_pts[l] = std::max(mg_max_pts[l], np);
                if (l >= 2) deep += np;
            }
            const int lc = G.mg_nlev - 1;
            mg_deep_pts = std::max(mg_deep_pts, deep);
            mg_coarse_pts = std::max(mg_coarse_pts, (long long)G.mg_lw[lc] * G.mg_lw[lc] * G.mg_lw[lc]);
        }
        if (G.p != 2) eoff += 6LL * G.n * G.n * G.n * NQ;
        voff += G.npts * R * C;
        doff += G.npts;
        qoff += (long long)G.ntiles * G.boxpts * R * C;
        max_pts = std::max(max_pts, G.npts);
        max_tets = std::max(max_tets, 6LL * G.n * G.n * G.n);
        max_tiles = std::max(max_tiles, G.ntiles);
        nr = std::max(nr, G.nrow);
    }
    W.total_vals = voff;
    W.total_pts = doff;
    W.total_q = qoff;
    Launch &L = W.L;
    const Launch old = L;
    L.nprob = nprob;
    L.nwg = nwg_override > 0 ? nwg_override
                              : (int)std::min<long long>(std::max<long long>((max_pts + 127) / 128, 1), 1024);
    L.max_tiles = max_tiles;
    L.nr = nr == 0 ? 0 : (nr == 1 ? 1 : 4);
    L.order = B->distinct[hp[0].geo]->geo.p;
    L.rg = L.order == 2 ? rg : R;   // orders 3, 4: all load cases in one workgroup
    L.max_tets = max_tets;
    L.total_q = qoff;
    W.nwg_gram = (int)std::min<long long>(std::max<long long>((max_pts + 4095) / 4096, 1), 256);
    W.nwg_avg = (int)std::min<long long>(std::max<long long>((max_tets + 1023) / 1024, 1), 256);
    const bool fp32 = B->opt.precision == CHOM_FP32_REFINED;
    const size_t nv = (size_t)voff, nq = (size_t)qoff;
    void *before[6] = {W.xd.p, W.xf.p, W.partial.p, W.probs.p, W.acc.p, W.accpq.p};
    CHOM_HIP(W.probs.ensure(nprob));
    if (eoff > 0) {
        CHOM_HIP(W.ef64.ensure((size_t)eoff));
        CHOM_HIP(W.ef32.ensure((size_t)eoff));
    }
    L.ef64 = eoff > 0 ? W.ef64.p : nullptr;
    L.ef32 = eoff > 0 ? W.ef32.p : nullptr;
    CHOM_HIP(W.b.ensure(nv));
    CHOM_HIP(W.q64.ensure(nq));
    CHOM_HIP(W.r64.ensure(nv));   // FP64 residual (refinement; final residual of the energy form)
    if (fp32) {
        CHOM_HIP(W.x64.ensure(nv));
        CHOM_HIP(W.xf.ensure(nv));
        CHOM_HIP(W.rf.ensure(nv));
        CHOM_HIP(W.pf.ensure(nv));
        CHOM_HIP(W.qf.ensure(nq));
        CHOM_HIP(W.r32.ensure(nv));
    } else {
        CHOM_HIP(W.xd.ensure(nv));
        CHOM_HIP(W.rd.ensure(nv));
        CHOM_HIP(W.pd.ensure(nv));
        CHOM_HIP(W.qd.ensure(nq));
    }
    CHOM_HIP(W.diag.ensure((size_t)doff * MS));
    CHOM_HIP(W.minv64.ensure((size_t)doff * MS));
    CHOM_HIP(W.minv32.ensure((size_t)doff * MS));
    const int S4 = C * 4;
    CHOM_HIP(W.ginv64.ensure((size_t)S4 * S4 * nprob));
    CHOM_HIP(W.ginv32.ensure((size_t)S4 * S4 * nprob));
    CHOM_HIP(W.ycoef.ensure((size_t)R * S4 * nprob));
    CHOM_HIP(W.cols.ensure((size_t)R * nprob));
    CHOM_HIP(W.cols_outer.ensure((size_t)R * nprob));
    CHOM_HIP(W.active.ensure(nprob));
    CHOM_HIP(W.active_outer.ensure(nprob));
    CHOM_HIP(W.bad.ensure(1));
    const int NC = (C == 3) ? 6 : 3;
    size_t part = 0;
    part = std::max(part, (size_t)nprob * L.nwg * R * (2 + C * 4));
    part = std::max(part, (size_t)nprob * L.max_tiles * R);
    part = std::max(part, (size_t)nprob * W.nwg_gram * 2 * 60);
    part = std::max(part, (size_t)nprob * W.nwg_avg * R * NC + (size_t)nprob * W.nwg_avg * R * R);
    part = std::max(part, (size_t)nprob * L.nwg * R * C * 4 + (size_t)nprob * R * C * 4);
    // two-level preconditioner
    Launch::Mg &M = L.mg;
    std::memset(&M, 0, sizeof(M));
    M.on = mg_nlev >= 2 ? 1 : 0;
    if (M.on) {
        constexpr int CC = C * C;
        M.nlev = mg_nlev;
        for (int l = 0; l < mg_nlev; ++l) {
            M.max_pts[l] = mg_max_pts[l];
            M.nwg[l] = (int)std::min<long long>(std::max<long long>((mg_max_pts[l] + 63) / 64, 1), 1024);
        }
        const char *sw = std::getenv("CHOM_MG_SWEEPS");
        M.sweeps = sw ? std::max(1, std::atoi(sw)) : 4;
        M.total_pts = moff;
        // LDS of the fused kernel: the four vectors of levels >= 2, then the coarsest stencils
        const long long tsz = fp32 ? (long long)sizeof(float) : (long long)sizeof(double);
        const long long vec_el = 4 * mg_deep_pts * C, sten_el = mg_coarse_pts * MG_SLOTS * CC;
        const long long budget = 60 * 1024;
        M.lds_vec = vec_el * tsz <= budget ? 1 : 0;
        M.lds_sten = (M.lds_vec && (vec_el + sten_el) * tsz <= budget) ? 1 : 0;
        M.lds_elems = (M.lds_vec ? vec_el : 0) + (M.lds_sten ? sten_el : 0);
        // FP32 and every coarsest level at depth 1, 2 or 3 with at most 512 points per level:
        // the up-front-load kernel (LDS: 3 level-2 vectors, 2 level-3 vectors, level-3 stencils and
        // inverses; on a level-1 coarsest the two iterates)
        M.small_elems = 0;
        M.small_bs = 512;
        if (fp32 && !std::getenv("CHOM_MG_GENERIC")) {
            long long need = 0, own = 0;
            bool ok = true;
            for (auto &P : hp) {
                const Geo &G = B->distinct[P.geo]->geo;
                if (G.mg_nlev < 2) continue;
                const int lc = G.mg_nlev - 1;
                if (lc == 1) {
                    const long long n1 = (long long)G.mg_lw[1] * G.mg_lw[1] * G.mg_lw[1];
                    if (n1 > 512) ok = false;
                    need = std::max(need, 2 * n1 * C);
                    own = std::max(own, n1);
                    continue;
                }
                const long long n2 = (long long)G.mg_lw[2] * G.mg_lw[2] * G.mg_lw[2];
                const long long n3 = lc == 3 ? (long long)G.mg_lw[3] * G.mg_lw[3] * G.mg_lw[3] : 0;
                if (lc > 3 || n2 > 512 || n3 > 512) ok = false;
                need = std::max(need, 3 * (n2 + 1) * C + 2 * (n3 + 1) * C + n3 * MG_SLOTS * CC + n3 * MS);
                own = std::max(own, std::max(n2, n3));
            }
            if (ok && need * (long long)sizeof(float) <= 64 * 1024) M.small_elems = need;
            const char *bs = std::getenv("CHOM_MG_SMALL_BS");
            M.small_bs = (own <= 256 && !(bs && std::atoi(bs) == 512)) ? 256 : 512;
        }
        const size_t np = (size_t)moff;
        CHOM_HIP(W.mgA64.ensure(np * MG_SLOTS * CC));
        CHOM_HIP(W.mgD64.ensure(np * MS));
        CHOM_HIP(W.mgrows1.ensure(np * 4));
        M.rows1 = W.mgrows1.p;
        CHOM_HIP(W.gmat.ensure((size_t)2 * nprob * (C * 4) * (C * 4)));
        CHOM_HIP(W.ginv_mg.ensure((size_t)nprob * (C * 4) * (C * 4)));
        M.A64 = W.mgA64.p;
        M.D64 = W.mgD64.p;
        if (fp32) {
            CHOM_HIP(W.mgA32.ensure(np * MG_SLOTS * CC));
            CHOM_HIP(W.mgD32.ensure(np * MS));
            CHOM_HIP(W.mgr32.ensure(np * R * C));
            CHOM_HIP(W.mgxp32.ensure(np * R * C));
            CHOM_HIP(W.mgres32.ensure(np * R * C));
            CHOM_HIP(W.mgx32.ensure(np * R * C));
            CHOM_HIP(W.mgW32.ensure(np * 4 * C * C));
            M.A = W.mgA32.p;
            M.Dinv = W.mgD32.p;
            M.r = W.mgr32.p;
            M.xp = W.mgxp32.p;
            M.res = W.mgres32.p;
            M.x = W.mgx32.p;
            M.W = W.mgW32.p;
        } else {
            CHOM_HIP(W.mgr64.ensure(np * R * C));
            CHOM_HIP(W.mgxp64.ensure(np * R * C));
            CHOM_HIP(W.mgres64.ensure(np * R * C));
            CHOM_HIP(W.mgx64.ensure(np * R * C));
            CHOM_HIP(W.mgW64.ensure(np * 4 * C * C));
            M.A = W.mgA64.p;
            M.Dinv = W.mgD64.p;
            M.r = W.mgr64.p;
            M.xp = W.mgxp64.p;
            M.res = W.mgres64.p;
            M.x = W.mgx64.p;
            M.W = W.mgW64.p;
        }
        part = std::max(part, (size_t)nprob * W.nwg_gram * 144);
    }
    CHOM_HIP(W.partial.ensure(part));
    {
        const size_t nacc = (size_t)nprob * R * ACC_RECMAX<C> * ACC_STRIPES, npq = (size_t)nprob * R * ACC_STRIPES;
        if (W.acc.n < nacc || W.accpq.n < npq) {
            CHOM_HIP(W.acc.ensure(nacc));
            CHOM_HIP(W.accpq.ensure(npq));
            CHOM_HIP(hipMemsetAsync(W.acc.p, 0, sizeof(double) * W.acc.n, W.stream));
            CHOM_HIP(hipMemsetAsync(W.accpq.p, 0, sizeof(double) * W.accpq.n, W.stream));
        }
    }
    CHOM_HIP(W.avg_out.ensure((size_t)nprob * R * NC));
    CHOM_HIP(W.avg_corr.ensure((size_t)nprob * R * NC));
    CHOM_HIP(W.cols_tmp.ensure((size_t)R * nprob));
    CHOM_HIP(W.cols_flush.ensure((size_t)R * nprob));
    CHOM_HIP(W.active_tmp.ensure(nprob));
    W.h_cols.resize((size_t)R * nprob);
    W.h_cols_outer.resize((size_t)R * nprob);
    W.h_cols_tmp.resize((size_t)R * nprob);
    CHOM_HIP(W.h_poll.ensure(nprob));
    W.refine_steps.assign(nprob, 0);
    L.geos = B->geos.p;
    L.probs = W.probs.p;
    const void *after[6] = {W.xd.p, W.xf.p, W.partial.p, W.probs.p, W.acc.p, W.accpq.p};
    if (std::memcmp(before, after, sizeof(before)) != 0 || old.nprob != L.nprob || old.nwg != L.nwg ||
        old.max_tiles != L.max_tiles || old.nr != L.nr || old.rg != L.rg ||
        std::memcmp(&old.mg, &L.mg, sizeof(L.mg)) != 0)
        ++W.gen;
    return CHOM_OK;
}

// A contiguous range of a class's problems solved as one CG chain: a launch
// restricted to the range (problem table offset, count) and the per-problem
// solver state of the range.  Vectors, tile boxes and coarse levels are
// addressed through the problems' own offsets, so chains over disjoint ranges
// share the class buffers and run concurrently on their own streams.
template <int C, int R> struct PcgChain {
    Launch L{};
    ColState *cols = nullptr;
    const ColState *mask = nullptr;
    int *active = nullptr;
    double *acc = nullptr, *accpq = nullptr, *ycoef = nullptr;
    const double *ginv = nullptr;
    long long acc_n = 0, accpq_n = 0;
    hipStream_t s = nullptr;
    GraphCache *graph = nullptr;
    int *h_active = nullptr;   // this chain's slice of the class's pinned poll buffer
    int max_iter = 0;          // CG steps per solve and column (0: no cap)
    ColState *cols_scratch = nullptr;   // this chain's slice of a scratch column buffer (compaction)
    double loose = 0.0;        // inner refinement passes: attainable-accuracy factor of the stopping test
};

template <int C, int R>
static PcgChain<C, R> make_chain(ClassWS<C, R> &W, int p0, int cnt, const double *ginv, const ColState *mask,
                                 hipStream_t s, GraphCache *graph) {
    constexpr int SMAX = C * 4;
    PcgChain<C, R> ch;
    ch.L = W.L;
    ch.L.probs = W.L.probs + p0;
    ch.L.nprob = cnt;
    ch.cols = W.cols.p + (size_t)p0 * R;
    ch.mask = mask ? mask + (size_t)p0 * R : nullptr;
    ch.active = W.active.p + p0;
    const long long accs = (long long)R * ACC_RECMAX<C> * ACC_STRIPES, pqs = (long long)R * ACC_STRIPES;
    ch.acc = W.acc.p + p0 * accs;
    ch.acc_n = cnt * accs;
    ch.accpq = W.accpq.p + p0 * pqs;
    ch.accpq_n = cnt * pqs;
    ch.ycoef = W.ycoef.p + (size_t)p0 * R * C * W.L.nr;
    ch.ginv = ginv + (size_t)p0 * SMAX * SMAX;
    ch.s = s;
    ch.graph = graph;
    ch.h_active = W.h_poll.p + p0;
    ch.cols_scratch = W.cols_flush.p + (size_t)p0 * R;
    return ch;
}

// One CG iteration (5 kernels, plus the V-cycle with the two-level preconditioner).
template <typename T, int C, int R>
static hipError_t cg_iteration(const PcgChain<C, R> &K, T *x, T *r, T *p, T *q, const void *minv, double rtol2,
                               int use_init) {
    const Launch &L = K.L;
    hipStream_t s = K.s;
    const bool mg = L.mg.on != 0;
    hipError_t e;
    if (mg && (e = launch_mg_fcorr<T, C, R>(L, K.ycoef, K.active, s)) != hipSuccess) return e;
    if ((e = launch_cg_dir<T, C, R>(L, x, r, p, minv, K.ycoef, K.cols, K.active, s, mg ? L.mg.res : nullptr,
                                    nullptr)) != hipSuccess)
        return e;
    if ((e = launch_operator<T, C, R>(L, L.nprob, L.rg, p, q, K.accpq, K.active, s)) != hipSuccess) return e;
    if ((e = launch_finish_alpha<C, R>(L, K.accpq, K.cols, s)) != hipSuccess) return e;
    if ((e = launch_cg_update<T, C, R>(L, r, q, minv, K.cols, K.acc, K.active, s)) != hipSuccess) return e;
    if (mg && (e = launch_mg_vcycle<T, C, R>(L, r, K.acc, K.active, s)) != hipSuccess) return e;
    return launch_finish_beta<C, R>(L, K.acc, K.ginv, K.ycoef, K.cols, K.active, 0, rtol2, use_init, nullptr, s,
                                    K.max_iter, nullptr, K.loose);
}

// Slot state of a chain that compaction permutes: problem table, column
// states, active counts, projection coefficients, Gram inverses (the vectors,
// tile boxes and coarse levels are addressed through the problem table).
template <int C, int R> struct ChainSlots {
    std::vector<Prob> pr;
    std::vector<ColState> cs;
    std::vector<int> act;
    std::vector<double> yc, gi;
};

template <int C, int R>
static int chain_download(const PcgChain<C, R> &K, int n, ChainSlots<C, R> &S) {
    const size_t ysz = (size_t)R * C * K.L.nr, gsz = (size_t)(4 * C) * (4 * C);
    S.pr.resize(n);
    S.cs.resize((size_t)n * R);
    S.act.resize(n);
    S.yc.resize((size_t)n * ysz);
    S.gi.resize((size_t)n * gsz);
    CHOM_HIP(hipMemcpyAsync(S.pr.data(), K.L.probs, sizeof(Prob) * n, hipMemcpyDeviceToHost, K.s));
    CHOM_HIP(hipMemcpyAsync(S.cs.data(), K.cols, sizeof(ColState) * n * R, hipMemcpyDeviceToHost, K.s));
    CHOM_HIP(hipMemcpyAsync(S.act.data(), K.active, sizeof(int) * n, hipMemcpyDeviceToHost, K.s));
    if (ysz) CHOM_HIP(hipMemcpyAsync(S.yc.data(), K.ycoef, sizeof(double) * n * ysz, hipMemcpyDeviceToHost, K.s));
    CHOM_HIP(hipMemcpyAsync(S.gi.data(), K.ginv, sizeof(double) * n * gsz, hipMemcpyDeviceToHost, K.s));
    CHOM_HIP(hipStreamSynchronize(K.s));
    return CHOM_OK;
}

// Writes the slots back in the order perm: new slot j takes old slot perm[j].
template <int C, int R>
static int chain_upload(const PcgChain<C, R> &K, const ChainSlots<C, R> &S, const std::vector<int> &perm) {
    const int n = (int)perm.size();
    const size_t ysz = (size_t)R * C * K.L.nr, gsz = (size_t)(4 * C) * (4 * C);
    ChainSlots<C, R> T;
    T.pr.resize(n);
    T.cs.resize((size_t)n * R);
    T.act.resize(n);
    T.yc.resize((size_t)n * ysz);
    T.gi.resize((size_t)n * gsz);
    for (int j = 0; j < n; ++j) {
        const int i = perm[j];
        T.pr[j] = S.pr[i];
        T.act[j] = S.act[i];
        for (int r = 0; r < R; ++r) T.cs[(size_t)j * R + r] = S.cs[(size_t)i * R + r];
        std::copy(S.yc.begin() + i * ysz, S.yc.begin() + (i + 1) * ysz, T.yc.begin() + j * ysz);
        std::copy(S.gi.begin() + i * gsz, S.gi.begin() + (i + 1) * gsz, T.gi.begin() + j * gsz);
    }
    CHOM_HIP(hipMemcpyAsync(const_cast<Prob *>(K.L.probs), T.pr.data(), sizeof(Prob) * n, hipMemcpyHostToDevice, K.s));
    CHOM_HIP(hipMemcpyAsync(K.cols, T.cs.data(), sizeof(ColState) * n * R, hipMemcpyHostToDevice, K.s));
    CHOM_HIP(hipMemcpyAsync(K.active, T.act.data(), sizeof(int) * n, hipMemcpyHostToDevice, K.s));
    if (ysz) CHOM_HIP(hipMemcpyAsync(K.ycoef, T.yc.data(), sizeof(double) * n * ysz, hipMemcpyHostToDevice, K.s));
    CHOM_HIP(hipMemcpyAsync(const_cast<double *>(K.ginv), T.gi.data(), sizeof(double) * n * gsz,
                            hipMemcpyHostToDevice, K.s));
    CHOM_HIP(hipStreamSynchronize(K.s));   // the host vectors die here
    return CHOM_OK;
}

// Compaction of a CG chain: when at most half of its problems are still active,
// the active ones move to the front of the chain's range and the launches shrink
// to them (problem count, tile count and coarse-level grids of those problems),
// so finished problems stop costing empty workgroups.  The pending x update of
// every leaving problem is applied first.  order[j]: original position of slot j.
template <typename T, int C, int R>
static int compact_chain(chom_batch *B, PcgChain<C, R> &K, T *x, const T *p, std::vector<int> &order) {
    const int n = K.L.nprob;
    ChainSlots<C, R> S;
    CHOM_TRY(chain_download<C, R>(K, n, S));
    std::vector<int> perm, leave;
    for (int i = 0; i < n; ++i) (S.act[i] ? perm : leave).push_back(i);
    const int nact = (int)perm.size();
    std::vector<ColState> fl(S.cs);
    for (int j = 0; j < nact; ++j)
        for (int r = 0; r < R; ++r) fl[(size_t)perm[j] * R + r].alpha = 0.0;
    CHOM_HIP(hipMemcpyAsync(K.cols_scratch, fl.data(), sizeof(ColState) * n * R, hipMemcpyHostToDevice, K.s));
    CHOM_HIP((launch_cg_flush_x<T, C, R>(K.L, x, p, K.cols_scratch, K.s)));
    for (int i : leave)
        for (int r = 0; r < R; ++r) S.cs[(size_t)i * R + r].alpha = 0.0;
    perm.insert(perm.end(), leave.begin(), leave.end());
    CHOM_TRY((chain_upload<C, R>(K, S, perm)));
    std::vector<int> o2(order.size());
    for (int j = 0; j < n; ++j) o2[j] = order[perm[j]];
    for (size_t j = n; j < order.size(); ++j) o2[j] = order[j];
    order.swap(o2);
    // launch shape of the remaining problems
    Launch &L = K.L;
    L.nprob = nact;
    int mt = 1;
    long long mp[MG_MAXLEV] = {};
    for (int j = 0; j < nact; ++j) {
        const Geo &G = B->distinct[S.pr[perm[j]].geo]->geo;
        mt = std::max(mt, G.ntiles);
        for (int l = 0; l < G.mg_nlev && l < MG_MAXLEV; ++l)
            mp[l] = std::max(mp[l], (long long)G.mg_lw[l] * G.mg_lw[l] * G.mg_lw[l]);
    }
    L.max_tiles = mt;
    if (L.mg.on)
        for (int l = 0; l < L.mg.nlev; ++l) {
            L.mg.max_pts[l] = mp[l];
            L.mg.nwg[l] = (int)std::min<long long>(std::max<long long>((mp[l] + 63) / 64, 1), 1024);
        }
    K.graph->reset();
    return CHOM_OK;
}

// PCG on one chain of problems: b -> x (vectors of precision T).  Iterations
// run in chunks, captured as a HIP graph and replayed; between chunks the host
// reads the per-problem active counts (finished problems cost only an early
// exit in every kernel) and compacts the chain when at most half of its
// problems remain (CHOM_NO_COMPACT turns that off); the slot order is restored
// at the end.
template <typename T, int C, int R>
static int pcg(chom_batch *B, ClassWS<C, R> &W, PcgChain<C, R> &K, const T *b, T *x, T *r, T *p, T *q,
               const void *minv, double rtol2, int use_init) {
    hipStream_t s = K.s;
    const Launch &L = K.L;
    const bool mg = L.mg.on != 0;
    GraphCache &GC = *K.graph;
    K.max_iter = B->opt.max_iter;
    // the accumulators may hold sums of kernels run outside a CG step (timing, residuals)
    CHOM_HIP(launch_zero(K.acc, K.acc_n, s));
    CHOM_HIP(launch_zero(K.accpq, K.accpq_n, s));
    CHOM_HIP((launch_cg_init<T, C, R>(L, b, x, r, minv, K.acc, s)));
    if (mg) CHOM_HIP((launch_mg_vcycle<T, C, R>(L, r, K.acc, nullptr, s)));
    CHOM_HIP((launch_finish_beta<C, R>(L, K.acc, K.ginv, K.ycoef, K.cols, K.active, 1, rtol2,
                                       K.mask ? 1 : use_init, K.mask, s, 0, nullptr, K.loose)));
    const int max_iter = B->opt.max_iter;
    const int chunk = 8;
    const bool use_graph = std::getenv("CHOM_NO_GRAPH") == nullptr;
    const bool compact = std::getenv("CHOM_NO_COMPACT") == nullptr;
    const int nfull = L.nprob;
    std::vector<int> order(nfull);
    for (int i = 0; i < nfull; ++i) order[i] = i;
    bool permuted = false;
    for (int it = 0; it < max_iter; it += chunk) {
        CHOM_HIP(hipMemcpyAsync(K.h_active, K.active, sizeof(int) * L.nprob, hipMemcpyDeviceToHost, s));
        CHOM_HIP(hipStreamSynchronize(s));
        int act = 0, nact = 0;
        for (int i = 0; i < L.nprob; ++i) {
            act += K.h_active[i];
            nact += K.h_active[i] ? 1 : 0;
        }
        if (act == 0) break;
        if (compact && L.nprob > 1 && 2 * nact <= L.nprob) {
            CHOM_TRY((compact_chain<T, C, R>(B, K, x, p, order)));
            permuted = true;
        }
        if (use_graph && (GC.exec == nullptr || GC.key != (const void *)x || GC.iters != chunk || GC.gen != W.gen ||
                          GC.probs != (const void *)L.probs || GC.nprob != L.nprob)) {
            GC.reset();
            hipGraph_t g;
            CHOM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            hipError_t ce = hipSuccess;
            for (int k = 0; k < chunk && ce == hipSuccess; ++k)
                ce = cg_iteration<T, C, R>(K, x, r, p, q, minv, rtol2, use_init);
            hipError_t ee = hipStreamEndCapture(s, &g);
            CHOM_HIP(ce);
            CHOM_HIP(ee);
            hipError_t ie = hipGraphInstantiate(&GC.exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            CHOM_HIP(ie);
            GC.key = x;
            GC.iters = chunk;
            GC.gen = W.gen;
            GC.probs = L.probs;
            GC.nprob = L.nprob;
        }
        if (use_graph) {
            CHOM_HIP(hipGraphLaunch(GC.exec, s));
        } else {
            for (int k = 0; k < chunk; ++k) CHOM_HIP((cg_iteration<T, C, R>(K, x, r, p, q, minv, rtol2, use_init)));
        }
    }
    // the last step's x += alpha p (every earlier one was applied by a direction kernel)
    CHOM_HIP((launch_cg_flush_x<T, C, R>(L, x, p, K.cols, s)));
    if (permuted) {   // back to the original slot order
        ChainSlots<C, R> S;
        CHOM_TRY((chain_download<C, R>(K, nfull, S)));
        std::vector<int> inv(nfull);
        for (int j = 0; j < nfull; ++j) inv[order[j]] = j;
        CHOM_TRY((chain_upload<C, R>(K, S, inv)));
        // the graph of the compacted chain no longer matches the problem table
        GC.reset();
    }
    return CHOM_OK;
}

// CG chains of a class.  Large classes (at least 16 problems) split into two
// chains of contiguous problem ranges, the second run from its own host thread
// on the class's second stream, so that the latency-bound kernels of one chain
// (coarse levels, finishing kernels, host polls) overlap the bandwidth- and
// ALU-bound ones of the other (512-record mixed batch: +4%); small classes keep
// one chain (the three-BC 24^3 batch: -8% with two).  CHOM_PCG_CHAINS=1 or 2
// forces the count.
static int chain_count(int nprob) {
    const char *ev = std::getenv("CHOM_PCG_CHAINS");
    const int want = ev ? std::atoi(ev) : (nprob >= 16 ? 2 : 1);
    return (nprob >= 2 && want == 2) ? 2 : 1;
}

// Runs fa() on the class's stream from this thread and fb() on its second
// stream from a host thread of its own.  The second stream first waits for the
// work already queued on the first; at the end the first waits for the second.
template <int C, int R, typename FA, typename FB>
static int fork_chains(ClassWS<C, R> &W, FA &&fa, FB &&fb) {
    hipEvent_t e0, e1;
    CHOM_HIP(hipEventCreateWithFlags(&e0, hipEventDisableTiming));
    CHOM_HIP(hipEventCreateWithFlags(&e1, hipEventDisableTiming));
    CHOM_HIP(hipEventRecord(e0, W.stream));
    CHOM_HIP(hipStreamWaitEvent(W.stream_b, e0, 0));
    int device = 0;
    CHOM_HIP(hipGetDevice(&device));
    int stb = CHOM_OK;
    std::string errb;
    std::thread th([&]() {
        if (hipSetDevice(device) != hipSuccess) {
            stb = CHOM_EDEVICE;
            errb = "hipSetDevice failed in a CG chain thread";
            return;
        }
        stb = fb();
        if (stb != CHOM_OK) errb = g_last_error;
    });
    const int sta = fa();
    th.join();
    hipError_t he = hipEventRecord(e1, W.stream_b);
    if (he == hipSuccess) he = hipStreamWaitEvent(W.stream, e1, 0);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (sta != CHOM_OK) return sta;
    if (stb != CHOM_OK) {
        set_error(errb);
        return stb;
    }
    CHOM_HIP(he);
    return CHOM_OK;
}

// PCG on all problems of a class, in one or two chains (chain_count).
template <typename T, int C, int R>
static int pcg_class(chom_batch *B, ClassWS<C, R> &W, bool fp64, const T *b, T *x, T *r, T *p, T *q,
                     const void *minv, const double *ginv, double rtol2, int use_init, const ColState *mask) {
    const int nprob = W.L.nprob;
    GraphCache *ga = fp64 ? &W.graph64 : &W.graph32, *gb = fp64 ? &W.graph64b : &W.graph32b;
    if (chain_count(nprob) == 1) {
        PcgChain<C, R> K = make_chain<C, R>(W, 0, nprob, ginv, mask, W.stream, ga);
        return pcg<T, C, R>(B, W, K, b, x, r, p, q, minv, rtol2, use_init);
    }
    const int h = (nprob + 1) / 2;
    PcgChain<C, R> KA = make_chain<C, R>(W, 0, h, ginv, mask, W.stream, ga);
    PcgChain<C, R> KB = make_chain<C, R>(W, h, nprob - h, ginv, mask, W.stream_b, gb);
    return fork_chains<C, R>(
        W, [&]() { return pcg<T, C, R>(B, W, KA, b, x, r, p, q, minv, rtol2, use_init); },
        [&]() { return pcg<T, C, R>(B, W, KB, b, x, r, p, q, minv, rtol2, use_init); });
}

// One CG chain's share of the FP32-operator / FP64-refinement solve: problems
// [p0, p0 + cnt), whose vector values are [v0, v1), on stream s with the
// chain's graph caches.  Each chain refines on its own, so neither waits for
// the other at a refinement step and one chain's FP64 residual and host checks
// overlap the other's CG.
template <int C, int R> struct RefineRange {
    int p0 = 0, cnt = 0;
    long long v0 = 0, v1 = 0;
    hipStream_t s = nullptr;
    GraphCache *g32 = nullptr, *g64 = nullptr;
};

// FP64 correction solve of the refinement for the problems of the range
// flagged in `which` (the others are masked out): K d = r64 with the FP64
// operator and block-Jacobi preconditioning to a tenth of the outer tolerance,
// then x64 += d.  Used when the FP32 inner solves stop contracting the FP64
// residual.  The FP64 vectors are allocated on first use (under alloc_mu: both
// chains may get here).
template <int C, int R>
static int fp64_correction(chom_batch *B, ClassWS<C, R> &W, const RefineRange<C, R> &G, const std::vector<int> &which,
                           double rtol2, std::mutex &alloc_mu) {
    const int nprob = W.L.nprob;
    const size_t c0 = (size_t)G.p0 * R, nc = (size_t)G.cnt * R;
    {
        std::lock_guard<std::mutex> lk(alloc_mu);
        const size_t nv = (size_t)W.total_vals, nq = (size_t)W.total_q;
        CHOM_HIP(W.xd.ensure(nv));
        CHOM_HIP(W.rd.ensure(nv));
        CHOM_HIP(W.pd.ensure(nv));
        CHOM_HIP(W.qd.ensure(nq));
        CHOM_HIP(W.cols_fb.ensure((size_t)R * nprob));
    }
    std::vector<ColState> mask(W.h_cols_outer.begin() + c0, W.h_cols_outer.begin() + c0 + nc);
    for (int i = 0; i < G.cnt; ++i)
        if (!which[i])
            for (int r = 0; r < R; ++r) mask[(size_t)i * R + r].done = COL_CONVERGED;
    CHOM_HIP(hipMemcpyAsync(W.cols_fb.p + c0, mask.data(), sizeof(ColState) * nc, hipMemcpyHostToDevice, G.s));
    PcgChain<C, R> K = make_chain<C, R>(W, G.p0, G.cnt, W.ginv64.p, W.cols_fb.p, G.s, G.g64);
    K.L.mg.on = 0;   // the coarse levels hold FP32 data in this mode: block Jacobi alone
    G.g64->reset();
    const int st = pcg<double, C, R>(B, W, K, W.r64.p, W.xd.p, W.rd.p, W.pd.p, W.qd.p, W.minv64.p, 0.01 * rtol2, 0);
    G.g64->reset();
    CHOM_TRY(st);
    CHOM_HIP(launch_axpy64(G.v1 - G.v0, W.x64.p + G.v0, W.xd.p + G.v0, G.s));
    CHOM_HIP(hipStreamSynchronize(G.s));   // mask dies here
    return CHOM_OK;
}

// FP32 operator with FP64 refinement on one range: x64 += PCG_32(r64),
// r64 = b - K_64 x64, until the projected FP64 residual meets rtol.  A problem
// whose FP64 residual norm contracts by less than a half per step over three
// steps is finished by an FP64 correction solve (CHOM_FORCE_FP64_FALLBACK
// forces that from the second step on, for tests).
template <int C, int R>
static int refine_range(chom_batch *B, ClassWS<C, R> &W, const RefineRange<C, R> &G, const double *ginv_inner32,
                        double rtol2, std::mutex &alloc_mu) {
    constexpr int SMAX = C * 4;
    const int p0 = G.p0, cnt = G.cnt;
    const size_t c0 = (size_t)p0 * R, nc = (size_t)cnt * R;
    hipStream_t s = G.s;
    Launch L = W.L;
    L.probs = W.L.probs + p0;
    L.nprob = cnt;
    const long long accs = (long long)R * ACC_RECMAX<C> * ACC_STRIPES;
    double *acc = W.acc.p + p0 * accs;
    const long long acc_n = cnt * accs;
    double *accpq = W.accpq.p + p0 * (long long)R * ACC_STRIPES;
    double *ycoef = W.ycoef.p + (size_t)p0 * R * C * L.nr;
    const double *ginv64 = W.ginv64.p + (size_t)p0 * SMAX * SMAX;
    const double *ginv32 = ginv_inner32 + (size_t)p0 * SMAX * SMAX;
    ColState *cols = W.cols.p + c0, *cols_outer = W.cols_outer.p + c0, *cols_tmp = W.cols_tmp.p + c0;
    int *active_outer = W.active_outer.p + p0, *active_tmp = W.active_tmp.p + p0;
    ColState *h_outer = W.h_cols_outer.data() + c0;
    const ColState *h_tmp = W.h_cols_tmp.data() + c0;
    const double irtol2 = B->opt.inner_rtol * B->opt.inner_rtol;
    const bool force_fb = std::getenv("CHOM_FORCE_FP64_FALLBACK") != nullptr;
    // An FP32 inner pass cannot resolve a column below about u32 * eref / E of
    // its own energy E (eref: the linear-field energy): the rounding of the
    // stiff phase's element contributions swamps the soft phase's where the
    // matrix is degraded.  Its stopping test is relaxed to that level (factor 6,
    // measured on the mixed batch between 1.5 and 100), so such a column stops
    // where FP32 stalls and the FP64 refinement continues from there.
    const double loose = 6.0 * 0x1p-24;
    const bool mg = L.mg.on != 0;
    std::vector<double> prev_rz(nc, 0.0);
    std::vector<int> slow(nc, 0);
    std::vector<ColState> fbmask;
    for (int step = 0; step <= B->opt.max_refine; ++step) {
        // outer residual: project r64 (FP64), then measure it in the metric of the
        // solver's preconditioner (r.M^-1 r, or r.B r with the two-level one, from
        // the FP32 copy with FP64 sums) against the column's energy
        CHOM_HIP(launch_zero(acc, acc_n, s));
        CHOM_HIP((launch_cg_init<double, C, R>(L, W.r64.p, nullptr, nullptr, W.minv64.p, acc, s)));
        CHOM_HIP((launch_finish_beta<C, R>(L, acc, ginv64, ycoef, cols_outer, active_outer, 1, rtol2, 0, nullptr, s,
                                           0, cols)));
        if (L.nr > 0) {
            CHOM_HIP((launch_proj_resid<C, R>(L, W.r64.p, W.r32.p, W.minv64.p, ycoef, acc, s)));
            CHOM_HIP((launch_finish_beta<C, R>(L, acc, ginv64, ycoef, cols_outer, active_outer, 1, rtol2, 0, nullptr,
                                               s, 0, cols)));
        }
        if (mg) {   // the two-level metric, into cols_tmp (merged on the host below)
            CHOM_HIP(hipMemcpyAsync(cols_tmp, cols_outer, sizeof(ColState) * nc, hipMemcpyDeviceToDevice, s));
            CHOM_HIP(launch_zero(acc, acc_n, s));
            CHOM_HIP((launch_cg_init<float, C, R>(L, W.r32.p, nullptr, nullptr, W.minv32.p, acc, s)));
            CHOM_HIP((launch_mg_vcycle<float, C, R>(L, W.r32.p, acc, nullptr, s)));
            CHOM_HIP((launch_finish_beta<C, R>(L, acc, ginv32, ycoef, cols_tmp, active_tmp, 1, rtol2, 0, nullptr, s,
                                               0, cols)));
            CHOM_HIP(hipMemcpyAsync(W.h_cols_tmp.data() + c0, cols_tmp, sizeof(ColState) * nc, hipMemcpyDeviceToHost,
                                    s));
        }
        CHOM_HIP(hipMemcpyAsync(h_outer, cols_outer, sizeof(ColState) * nc, hipMemcpyDeviceToHost, s));
        CHOM_HIP(hipStreamSynchronize(s));
        // merge: the two-level measurement where it is finite; where the FP32
        // coarse levels overflow, the FP64 block-Jacobi one stands and an active
        // column goes to the FP64 correction solve
        std::vector<int> fp32_failed(cnt, 0);
        if (mg) {
            for (size_t k = 0; k < nc; ++k) {
                ColState &h = h_outer[k];
                const ColState &t = h_tmp[k];
                if (std::isfinite(t.rz)) {
                    if (h.done != COL_NONFINITE) {
                        h.rz = t.rz;
                        h.rz_init = t.rz_init;
                        h.done = t.done;
                    }
                } else if (h.done == COL_ACTIVE) {
                    fp32_failed[k / R] = 1;
                }
            }
            CHOM_HIP(hipMemcpyAsync(cols_outer, h_outer, sizeof(ColState) * nc, hipMemcpyHostToDevice, s));
        }
        int act = 0;
        std::vector<int> stalled(cnt, 0);
        bool any_stalled = false;
        for (int i = 0; i < cnt; ++i) {
            int active = 0;
            for (int r = 0; r < R; ++r) active += h_outer[(size_t)i * R + r].done == COL_ACTIVE;
            act += active;
            if (!active) continue;
            W.refine_steps[p0 + i] = step;
            if (fp32_failed[i]) stalled[i] = 1;
            for (int r = 0; r < R; ++r) {
                const size_t k = (size_t)i * R + r;
                const ColState &cs = h_outer[k];
                if (cs.done) continue;
                const bool contracted = step > 0 && cs.rz <= 0.25 * prev_rz[k];
                slow[k] = (step > 0 && !contracted) ? slow[k] + 1 : 0;
                if (slow[k] >= 3 || (force_fb && step >= 1)) stalled[i] = 1;
                prev_rz[k] = cs.rz;
            }
            if (stalled[i]) {
                any_stalled = true;
                W.fallback[p0 + i] = 1;
                for (int r = 0; r < R; ++r) slow[(size_t)i * R + r] = 0;
            }
        }
        if (act == 0 || step == B->opt.max_refine) break;
        if (any_stalled) {
            CHOM_TRY((fp64_correction<C, R>(B, W, G, stalled, rtol2, alloc_mu)));
            // the other active problems still take their FP32 correction this step
            fbmask.assign(h_outer, h_outer + nc);
            for (int i = 0; i < cnt; ++i)
                if (stalled[i])
                    for (int r = 0; r < R; ++r) fbmask[(size_t)i * R + r].done = COL_CONVERGED;
            CHOM_HIP(hipMemcpyAsync(W.cols_fb.p + c0, fbmask.data(), sizeof(ColState) * nc, hipMemcpyHostToDevice, s));
        }
        PcgChain<C, R> K = make_chain<C, R>(W, p0, cnt, ginv_inner32, any_stalled ? W.cols_fb.p : W.cols_outer.p, s,
                                            G.g32);
        K.loose = loose;
        CHOM_TRY((pcg<float, C, R>(B, W, K, W.r32.p, W.xf.p, W.rf.p, W.pf.p, W.qf.p, W.minv32.p, irtol2, 1)));
        CHOM_HIP(launch_axpy_x64(G.v1 - G.v0, W.x64.p + G.v0, W.xf.p + G.v0, s));
        CHOM_HIP((launch_operator<double, C, R>(L, cnt, L.rg, W.x64.p, W.q64.p, accpq, nullptr, s)));
        CHOM_HIP((launch_residual64<C, R>(L, W.b.p, W.q64.p, W.r64.p, W.r32.p, s)));
    }
    return CHOM_OK;
}

// FP32 operator with FP64 refinement for a class: x64 = 0, r64 = b, then the
// refinement per CG chain (chain_count), each chain on its own problem range.
template <int C, int R>
static int refine_class(chom_batch *B, ClassWS<C, R> &W, const std::vector<Prob> &hprobs,
                        const double *ginv_inner32, double rtol2) {
    const int nprob = W.L.nprob;
    hipStream_t s = W.stream;
    CHOM_HIP(hipMemsetAsync(W.x64.p, 0, sizeof(double) * W.total_vals, s));
    CHOM_HIP((launch_residual64<C, R>(W.L, W.b.p, nullptr, W.r64.p, W.r32.p, s)));
    CHOM_HIP(hipMemcpyAsync(W.cols_outer.p, W.cols.p, sizeof(ColState) * R * nprob, hipMemcpyDeviceToDevice, s));
    std::mutex alloc_mu;
    if (chain_count(nprob) == 1) {
        const RefineRange<C, R> G{0, nprob, 0, W.total_vals, s, &W.graph32, &W.graph64};
        return refine_range<C, R>(B, W, G, ginv_inner32, rtol2, alloc_mu);
    }
    const int h = (nprob + 1) / 2;
    const long long vh = hprobs[h].voff;
    const RefineRange<C, R> GA{0, h, 0, vh, s, &W.graph32, &W.graph64};
    const RefineRange<C, R> GB{h, nprob - h, vh, W.total_vals, W.stream_b, &W.graph32b, &W.graph64b};
    return fork_chains<C, R>(
        W, [&]() { return refine_range<C, R>(B, W, GA, ginv_inner32, rtol2, alloc_mu); },
        [&]() { return refine_range<C, R>(B, W, GB, ginv_inner32, rtol2, alloc_mu); });
}

// Solve one class (mechanical or scalar) for all its problems.  Result: W.avg_out.
template <int C, int R>
static int run_class(chom_batch *B, ClassWS<C, R> &W, std::vector<Prob> &hprobs, int rg, int nwg) {
    hipStream_t s = W.stream;
    CHOM_TRY((setup_class<C, R>(B, W, hprobs, rg, nwg)));
    const Launch &L = W.L;
    const int nprob = L.nprob;
    CHOM_HIP(hipMemcpyAsync(W.probs.p, hprobs.data(), sizeof(Prob) * nprob, hipMemcpyHostToDevice, s));
    CHOM_HIP(hipMemsetAsync(W.cols.p, 0, sizeof(ColState) * R * nprob, s));
    CHOM_HIP(hipMemsetAsync(W.bad.p, 0, sizeof(int), s));
    if (L.order != 2) CHOM_HIP((launch_factors_hp<C>(L, W.ef64.p, W.ef32.p, s)));
    CHOM_HIP((launch_precond<C>(L, W.total_pts, W.diag.p, W.minv64.p, W.minv32.p, W.q64.p, s)));
    const bool mg = L.mg.on != 0;
    CHOM_HIP((launch_gram<C>(L, W.minv64.p, W.minv32.p, W.partial.p, W.nwg_gram, W.ginv64.p, W.ginv32.p, W.bad.p, s,
                             mg ? W.gmat.p : nullptr)));
    const double *ginv_inner64 = W.ginv64.p, *ginv_inner32 = W.ginv32.p;
    if (mg) {
        const size_t SS = (size_t)(C * 4) * (C * 4);
        if (B->opt.precision == CHOM_FP64) {
            CHOM_HIP((launch_mg_stencils<double, C>(L, (double *)nullptr, (double *)nullptr, s)));
            CHOM_HIP((launch_mg_gram<double, C, R>(L, W.pd.p, W.gmat.p, W.partial.p, W.nwg_gram, W.ginv_mg.p,
                                                   W.bad.p, s)));
            ginv_inner64 = W.ginv_mg.p;
        } else {
            CHOM_HIP((launch_mg_stencils<float, C>(L, W.mgA32.p, W.mgD32.p, s)));
            CHOM_HIP((launch_mg_gram<float, C, R>(L, W.pf.p, W.gmat.p + SS * nprob, W.partial.p, W.nwg_gram,
                                                  W.ginv_mg.p, W.bad.p, s)));
            ginv_inner32 = W.ginv_mg.p;
        }
    }
    CHOM_HIP((launch_rhs<C, R>(L, W.total_vals, W.b.p, W.cols.p, W.q64.p, W.accpq.p, s)));
    const double rtol2 = B->opt.rtol * B->opt.rtol;
    W.fallback.assign(nprob, 0);
    double *x64 = nullptr;
    if (B->opt.precision == CHOM_FP64) {
        CHOM_TRY((pcg_class<double, C, R>(B, W, true, W.b.p, W.xd.p, W.rd.p, W.pd.p, W.qd.p, W.minv64.p,
                                          ginv_inner64, rtol2, 0, nullptr)));
        x64 = W.xd.p;
    } else {
        CHOM_TRY((refine_class<C, R>(B, W, hprobs, ginv_inner32, rtol2)));
        x64 = W.x64.p;
    }
    CHOM_HIP((launch_project<C, R>(L, x64, W.minv64.p, W.ginv64.p, W.partial.p, s)));
    // residual of the projected solution, r = b - K x (FP64 operator), itself
    // projected: the energy form of the averages and the Hill-Mandel gap take it
    CHOM_HIP((launch_operator<double, C, R>(L, nprob, L.rg, x64, W.q64.p, W.accpq.p, nullptr, s)));
    CHOM_HIP((launch_residual64<C, R>(L, W.b.p, W.q64.p, W.r64.p, nullptr, s)));
    if (L.nr > 0) {
        CHOM_HIP(hipMemsetAsync(W.cols_tmp.p, 0, sizeof(ColState) * R * nprob, s));
        CHOM_HIP(launch_zero(W.acc.p, (long long)W.acc.n, s));
        CHOM_HIP((launch_cg_init<double, C, R>(L, W.r64.p, nullptr, nullptr, W.minv64.p, W.acc.p, s)));
        CHOM_HIP((launch_finish_beta<C, R>(L, W.acc.p, W.ginv64.p, W.ycoef.p, W.cols_tmp.p, W.active_tmp.p, 1, rtol2,
                                           0, nullptr, s)));
        CHOM_HIP((launch_proj_resid<C, R>(L, W.r64.p, nullptr, W.minv64.p, W.ycoef.p, W.acc.p, s)));
        CHOM_HIP(launch_zero(W.acc.p, (long long)W.acc.n, s));
    }
    CHOM_HIP(launch_zero(W.accpq.p, (long long)W.accpq.n, s));
    CHOM_HIP((launch_average<C, R>(L, x64, W.r64.p, W.partial.p, W.nwg_avg, W.avg_out.p, s, W.avg_corr.p)));
    CHOM_HIP(hipMemcpyAsync(W.h_cols.data(), W.cols.p, sizeof(ColState) * R * nprob, hipMemcpyDeviceToHost, s));
    if (B->opt.precision == CHOM_FP32_REFINED)
        CHOM_HIP(hipMemcpyAsync(W.h_cols_outer.data(), W.cols_outer.p, sizeof(ColState) * R * nprob,
                                hipMemcpyDeviceToHost, s));
    int hbad = 0;
    CHOM_HIP(hipMemcpyAsync(&hbad, W.bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
    CHOM_HIP(hipStreamSynchronize(s));
    if (hbad) {
        set_error("constraint Gram matrix singular");
        return CHOM_EDEVICE;
    }
    return CHOM_OK;
}

// Time `reps` operator launches of a class with load-case grouping rg (ms per launch).
template <typename T, int C, int R>
static int time_op(chom_batch *B, ClassWS<C, R> &W, const T *x, T *y, int rg, int reps, double *ms) {
    const Launch &L = W.L;
    hipStream_t s = W.stream;
    hipEvent_t e0, e1;
    CHOM_HIP(hipEventCreate(&e0));
    CHOM_HIP(hipEventCreate(&e1));
    CHOM_HIP((launch_operator<T, C, R>(L, L.nprob, rg, x, y, W.accpq.p, nullptr, s)));
    CHOM_HIP(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i)
        CHOM_HIP((launch_operator<T, C, R>(L, L.nprob, rg, x, y, W.accpq.p, nullptr, s)));
    CHOM_HIP(hipEventRecord(e1, s));
    CHOM_HIP(hipEventSynchronize(e1));
    float t = 0.f;
    CHOM_HIP(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = (double)t / reps;
    return CHOM_OK;
}

// Time `reps` CG vector sweeps (dir + update) with nwg workgroups per problem.
template <typename T, int C, int R>
static int time_vec(chom_batch *B, ClassWS<C, R> &W, T *x, T *r, T *p, const T *q, const void *minv, int nwg,
                    int reps, double *ms) {
    Launch L = W.L;
    L.nwg = nwg;
    hipStream_t s = W.stream;
    std::vector<int> ones(L.nprob, 1);
    CHOM_HIP(hipMemcpyAsync(W.active.p, ones.data(), sizeof(int) * L.nprob, hipMemcpyHostToDevice, s));
    CHOM_HIP(hipMemsetAsync(W.cols.p, 0, sizeof(ColState) * R * L.nprob, s));
    hipEvent_t e0, e1;
    CHOM_HIP(hipEventCreate(&e0));
    CHOM_HIP(hipEventCreate(&e1));
    CHOM_HIP(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i) {
        CHOM_HIP((launch_cg_dir<T, C, R>(L, x, r, p, minv, W.ycoef.p, W.cols.p, W.active.p, s)));
        CHOM_HIP((launch_cg_update<T, C, R>(L, r, q, minv, W.cols.p, W.acc.p, W.active.p, s)));
    }
    CHOM_HIP(hipEventRecord(e1, s));
    CHOM_HIP(hipEventSynchronize(e1));
    float t = 0.f;
    CHOM_HIP(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    CHOM_HIP(hipStreamSynchronize(s));
    *ms = (double)t / reps;
    return CHOM_OK;
}

// Autotune one class: operator grouping rg and vector workgroups per problem,
// timed on the batch's own problem table with zero operands (the cost of these
// kernels does not depend on the values).
template <int C, int R>
static int autotune_class(chom_batch *B, ClassWS<C, R> &W, std::vector<Prob> &hp, const std::string &key,
                          int *rg_out, int *nwg_out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load();
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
        *rg_out = it->second.first;
        *nwg_out = it->second.second;
        return CHOM_OK;
    }
    CHOM_TRY((setup_class<C, R>(B, W, hp, *rg_out, 1024)));   // partials sized for the largest candidate
    hipStream_t s = W.stream;
    CHOM_HIP(hipMemcpyAsync(W.probs.p, hp.data(), sizeof(Prob) * hp.size(), hipMemcpyHostToDevice, s));
    const bool f32 = B->opt.precision == CHOM_FP32_REFINED;
    const size_t nv = W.total_vals, nq = W.total_q;
    if (f32) {
        CHOM_HIP(hipMemsetAsync(W.pf.p, 0, sizeof(float) * nv, s));
        CHOM_HIP(hipMemsetAsync(W.rf.p, 0, sizeof(float) * nv, s));
        CHOM_HIP(hipMemsetAsync(W.xf.p, 0, sizeof(float) * nv, s));
        CHOM_HIP(hipMemsetAsync(W.qf.p, 0, sizeof(float) * nq, s));
        CHOM_HIP(hipMemsetAsync(W.minv32.p, 0, sizeof(float) * W.total_pts * ClassWS<C, R>::MS, s));
    } else {
        CHOM_HIP(hipMemsetAsync(W.pd.p, 0, sizeof(double) * nv, s));
        CHOM_HIP(hipMemsetAsync(W.rd.p, 0, sizeof(double) * nv, s));
        CHOM_HIP(hipMemsetAsync(W.xd.p, 0, sizeof(double) * nv, s));
        CHOM_HIP(hipMemsetAsync(W.qd.p, 0, sizeof(double) * nq, s));
        CHOM_HIP(hipMemsetAsync(W.minv64.p, 0, sizeof(double) * W.total_pts * ClassWS<C, R>::MS, s));
    }
    CHOM_HIP(hipMemsetAsync(W.ycoef.p, 0, sizeof(double) * W.ycoef.n, s));
    const int rgs_mech[3] = {1, 2, 3}, rgs_scal[2] = {1, 3};
    const int *rgs = (C == 3) ? rgs_mech : rgs_scal;
    const int nrg = W.L.order != 2 ? 0 : (C == 3) ? 3 : 2;   // orders 3, 4 always take all load cases
    double best = 1e30;
    int best_rg = W.L.order == 2 ? *rg_out : R;
    for (int i = 0; i < nrg; ++i) {
        double ms;
        if (f32) CHOM_TRY((time_op<float, C, R>(B, W, W.pf.p, W.qf.p, rgs[i], 5, &ms)));
        else CHOM_TRY((time_op<double, C, R>(B, W, W.pd.p, W.qd.p, rgs[i], 5, &ms)));
        if (ms < best) {
            best = ms;
            best_rg = rgs[i];
        }
    }
    W.L.rg = best_rg;
    const int nwgs[4] = {128, 256, 512, 1024};
    best = 1e30;
    int best_nwg = W.L.nwg;
    for (int i = 0; i < 4; ++i) {
        double ms;
        if (f32) CHOM_TRY((time_vec<float, C, R>(B, W, W.xf.p, W.rf.p, W.pf.p, W.qf.p, W.minv32.p, nwgs[i], 5, &ms)));
        else CHOM_TRY((time_vec<double, C, R>(B, W, W.xd.p, W.rd.p, W.pd.p, W.qd.p, W.minv64.p, nwgs[i], 5, &ms)));
        if (ms < best) {
            best = ms;
            best_nwg = nwgs[i];
        }
    }
    *rg_out = best_rg;
    *nwg_out = best_nwg;
    tune_store(key, best_rg, best_nwg);
    return CHOM_OK;
}

static std::string tune_key(chom_batch *B, int physics) {
    hipDeviceProp_t prop;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::string name = "gpu";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) name = prop.gcnArchName;
    for (auto &ch : name)
        if (ch == ' ' || ch == ':') ch = '_';
    std::string key = name + "/" + (physics == 0 ? "mech" : "scal") + "/" +
                      (B->opt.precision == CHOM_FP32_REFINED ? "f32" : "f64") + "/p" +
                      std::to_string(B->distinct.empty() ? 2 : B->distinct[0]->order) + "/";
    std::map<std::pair<int, int>, int> sizes;
    for (auto *r : B->entries) sizes[{r->n, r->bc}] += 1;
    for (auto &kv : sizes)
        key += std::to_string(kv.first.first) + "b" + std::to_string(kv.first.second) + "x" + std::to_string(kv.second) + ",";
    return key;
}

// ------------------------------------------------------------------ batch solve
static int batch_init(chom_batch *B, chom_rve *const *rves, int n, const chom_options *opt) {
    B->entries.assign(rves, rves + n);
    std::map<chom_rve *, int> idx;
    for (int i = 0; i < n; ++i) {
        auto it = idx.find(rves[i]);
        if (it == idx.end()) {
            const int k = (int)B->distinct.size();
            idx[rves[i]] = k;
            B->distinct.push_back(rves[i]);
            B->geo_of.push_back(k);
        } else {
            B->geo_of.push_back(it->second);
        }
    }
    for (auto *r : B->distinct)
        if (r->order != B->distinct[0]->order) {
            set_error("chom_batch_create: all RVEs of a batch must have the same order");
            return CHOM_EINVAL;
        }
    B->opt = *opt;
    if (B->opt.hip_stream) {
        B->stream = (hipStream_t)B->opt.hip_stream;
    } else {
        CHOM_HIP(hipStreamCreate(&B->stream));   // default priority
        B->own_stream = true;
    }
    CHOM_HIP(hipStreamCreate(&B->stream2));      // default priority
    B->mech.stream = B->stream;
    B->scal.stream = B->stream2;
    CHOM_HIP(hipStreamCreate(&B->mech.stream_b));   // second CG chain of each class, default priority
    CHOM_HIP(hipStreamCreate(&B->scal.stream_b));
    std::vector<Geo> hg;
    for (auto *r : B->distinct) hg.push_back(r->geo);
    CHOM_HIP(B->geos.ensure(hg.size()));
    CHOM_HIP(hipMemcpyAsync(B->geos.p, hg.data(), sizeof(Geo) * hg.size(), hipMemcpyHostToDevice, B->stream));
    CHOM_HIP(hipStreamSynchronize(B->stream));
    return CHOM_OK;
}

// Cholesky test of a symmetric n x n matrix (row-major): true if positive definite.
static bool cholesky_ok(const double *A, int n) {
    double L[36];
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        L[j * n + j] = std::sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            double v = A[i * n + j];
            for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = v / L[j * n + j];
        }
    }
    return true;
}

static double fro_ratio(const double *num, const double *den, int n) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < n; ++k) {
        a += num[k] * num[k];
        b += den[k] * den[k];
    }
    return b > 0.0 ? std::sqrt(a / b) : 0.0;
}

static int batch_homogenise(chom_batch *B, const chom_params *params, double *C_hom, double *K_hom, double *D_hom,
                            chom_report *rep, bool dev) {
    const int batch = (int)B->entries.size();
    hipStream_t s = B->stream;
    std::vector<chom_params> hp(batch);
    if (dev)
        CHOM_HIP(hipMemcpy(hp.data(), params, sizeof(chom_params) * batch, hipMemcpyDeviceToHost));
    else
        std::memcpy(hp.data(), params, sizeof(chom_params) * batch);
    std::vector<Prob> pm(batch), ps(2 * batch);
    std::vector<double> keep(batch);
    const bool sweeps_env = std::getenv("CHOM_MG_SWEEPS") != nullptr;
    for (int i = 0; i < batch; ++i) {
        chom_rve *rv = B->entries[i];
        double m10[10], t4[4], d4[4];
        const int st = material_constants(&rv->mat, &hp[i], B->opt.c_sat, B->opt.degrade_yarn, m10, t4, d4, &keep[i]);
        if (st != CHOM_OK) {
            set_error(std::string("record ") + std::to_string(i) + ": " + g_last_error);
            return st;
        }
        std::memset(&pm[i], 0, sizeof(Prob));
        std::memset(&ps[i], 0, sizeof(Prob));
        std::memset(&ps[batch + i], 0, sizeof(Prob));
        for (int ph = 0; ph < 2; ++ph)
            for (int k = 0; k < 5; ++k) {
                pm[i].mat64[ph][k] = m10[5 * ph + k];
                pm[i].mat32[ph][k] = (float)m10[5 * ph + k];
            }
        for (int ph = 0; ph < 2; ++ph)
            for (int k = 0; k < 2; ++k) {
                ps[i].mat64[ph][k] = t4[2 * ph + k];
                ps[i].mat32[ph][k] = (float)t4[2 * ph + k];
                ps[batch + i].mat64[ph][k] = d4[2 * ph + k];
                ps[batch + i].mat32[ph][k] = (float)d4[2 * ph + k];
            }
        pm[i].geo = ps[i].geo = ps[batch + i].geo = B->geo_of[i];
        // Coarsest-level sweeps of the mechanical problem: the coarsest level carries
        // the soft modes of a degraded matrix, so a record whose yarn-to-matrix shear
        // modulus ratio exceeds 10 (about 3.3 undegraded: (1 - omega) below about
        // 1/3) takes 32 sweeps there instead of the class's 4 (CHOM_MG_SWEEPS
        // overrides both).  Measured on the mixed batch: 416 -> 459
        // homogenisations/s, the undegraded 24^3 batch unchanged; thresholds 10 to
        // 100 and 32 to 64 sweeps within 0.5%.
        const double ratio = m10[6] / std::max(m10[1], 1e-300);
        if (!sweeps_env) pm[i].mg_sweeps = ratio > 10.0 ? 32 : 0;
        // The per-column energy test bounds each column's error, not C_bar's softest
        // directions, whose share of a stiff column's energy falls with the
        // yarn/matrix contrast: past a shear-modulus ratio of 3e4 ((1 - omega) below
        // about 1e-4) the mechanical stopping tests tighten rtol^2 by 3e4 / ratio
        // (the benchmark's records stay below that ratio and are untouched).
        pm[i].rtol2_scale = ratio > 3e4 ? 3e4 / ratio : 1.0;
    }
    if (!B->tuned && std::getenv("CHOM_AUTOTUNE")) {
        CHOM_TRY((autotune_class<3, 6>(B, B->mech, pm, tune_key(B, 0), &B->rg_mech, &B->nwg_mech)));
        CHOM_TRY((autotune_class<1, 3>(B, B->scal, ps, tune_key(B, 1), &B->rg_scal, &B->nwg_scal)));
        B->tuned = true;
    }
    // the two classes are independent: the scalar one runs on its own stream from
    // a second host thread (its host loops then overlap the mechanical ones)
    {
        hipEvent_t ev;
        CHOM_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        CHOM_HIP(hipEventRecord(ev, s));
        CHOM_HIP(hipStreamWaitEvent(B->stream2, ev, 0));
        (void)hipEventDestroy(ev);
    }
    int device = 0;
    CHOM_HIP(hipGetDevice(&device));
    int st_scal = CHOM_OK;
    std::string err_scal;
    const bool serial = std::getenv("CHOM_SERIAL_CLASSES") != nullptr;
    auto scal_job = [&]() {
        if (hipSetDevice(device) != hipSuccess) {
            st_scal = CHOM_EDEVICE;
            err_scal = "hipSetDevice failed in the scalar-class thread";
            return;
        }
        st_scal = run_class<1, 3>(B, B->scal, ps, B->rg_scal, B->nwg_scal);
        if (st_scal != CHOM_OK) err_scal = g_last_error;
    };
    int st_mech = CHOM_OK;
    if (serial) {
        st_mech = run_class<3, 6>(B, B->mech, pm, B->rg_mech, B->nwg_mech);
        if (st_mech == CHOM_OK) scal_job();
    } else {
        std::thread th(scal_job);
        st_mech = run_class<3, 6>(B, B->mech, pm, B->rg_mech, B->nwg_mech);
        th.join();
    }
    if (st_mech != CHOM_OK) return st_mech;
    if (st_scal != CHOM_OK) {
        set_error(err_scal);
        return st_scal;
    }
    std::vector<double> cm((size_t)batch * 36), cs((size_t)2 * batch * 9);
    std::vector<double> gm((size_t)batch * 36), gs((size_t)2 * batch * 9);
    CHOM_HIP(hipMemcpyAsync(cm.data(), B->mech.avg_out.p, sizeof(double) * cm.size(), hipMemcpyDeviceToHost, s));
    CHOM_HIP(hipMemcpyAsync(gm.data(), B->mech.avg_corr.p, sizeof(double) * gm.size(), hipMemcpyDeviceToHost, s));
    CHOM_HIP(hipMemcpyAsync(cs.data(), B->scal.avg_out.p, sizeof(double) * cs.size(), hipMemcpyDeviceToHost,
                            B->stream2));
    CHOM_HIP(hipMemcpyAsync(gs.data(), B->scal.avg_corr.p, sizeof(double) * gs.size(), hipMemcpyDeviceToHost,
                            B->stream2));
    CHOM_HIP(hipStreamSynchronize(B->stream2));
    CHOM_HIP(hipStreamSynchronize(s));
    std::vector<double> oc((size_t)batch * 21), ok((size_t)batch * 6), od((size_t)batch * 6);
    int overall = CHOM_OK;
    const bool refined = B->opt.precision == CHOM_FP32_REFINED;
    for (int i = 0; i < batch; ++i) {
        const double *Cm = &cm[(size_t)i * 36];
        int q = 0;
        double fro = 0, asym = 0;
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) {
                if (b >= a) oc[(size_t)i * 21 + q++] = Cm[a * 6 + b];
                fro += Cm[a * 6 + b] * Cm[a * 6 + b];
                const double dlt = Cm[a * 6 + b] - Cm[b * 6 + a];
                asym += dlt * dlt;
            }
        const double *Kt = &cs[(size_t)i * 9], *Dt = &cs[(size_t)(batch + i) * 9];
        const int ui[6] = {0, 4, 8, 1, 5, 2};
        for (int k = 0; k < 6; ++k) {
            ok[(size_t)i * 6 + k] = Kt[ui[k]];
            od[(size_t)i * 6 + k] = Dt[ui[k]];
        }
        chom_report Rp;
        std::memset(&Rp, 0, sizeof(Rp));
        Rp.status = CHOM_OK;
        Rp.asym = fro > 0 ? std::sqrt(asym / fro) : 0.0;
        Rp.omega_keep = keep[i];
        for (int c = 0; c < 12; ++c) {
            const ColState *cin, *cout;
            if (c < 6) {
                cin = &B->mech.h_cols[(size_t)i * 6 + c];
                cout = refined ? &B->mech.h_cols_outer[(size_t)i * 6 + c] : cin;
            } else {
                const int pidx = (c < 9) ? i : batch + i;
                const int ridx = (c < 9) ? c - 6 : c - 9;
                cin = &B->scal.h_cols[(size_t)pidx * 3 + ridx];
                cout = refined ? &B->scal.h_cols_outer[(size_t)pidx * 3 + ridx] : cin;
            }
            Rp.iters[c] = cin->iters;
            Rp.resid[c] = cout->eref > 0 ? std::sqrt(cout->rz / cout->eref) : 0.0;
            const bool finite = std::isfinite(cout->rz) && cout->done != COL_NONFINITE && cin->done != COL_NONFINITE;
            const bool conv = finite && cout->done == COL_CONVERGED;
            if (!conv) {
                Rp.status = CHOM_ENOCONV;
                Rp.fail[c] = !finite ? CHOM_FAIL_NONFINITE
                                     : (cout->done == COL_BREAKDOWN || cin->done == COL_BREAKDOWN) ? CHOM_FAIL_BREAKDOWN
                                                                                                  : CHOM_FAIL_CAP;
            }
        }
        if (refined) {
            Rp.refine_steps[0] = B->mech.refine_steps[i];
            Rp.refine_steps[1] = B->scal.refine_steps[i];
            Rp.refine_steps[2] = B->scal.refine_steps[batch + i];
            Rp.fp64_fallback[0] = B->mech.fallback[i];
            Rp.fp64_fallback[1] = B->scal.fallback[i];
            Rp.fp64_fallback[2] = B->scal.fallback[batch + i];
        }
        // positive definiteness of the symmetric parts, and the Hill-Mandel gap
        {
            double S6[36], S3k[9], S3d[9];
            for (int a = 0; a < 6; ++a)
                for (int b = 0; b < 6; ++b) S6[a * 6 + b] = 0.5 * (Cm[a * 6 + b] + Cm[b * 6 + a]);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    S3k[a * 3 + b] = 0.5 * (Kt[a * 3 + b] + Kt[b * 3 + a]);
                    S3d[a * 3 + b] = 0.5 * (Dt[a * 3 + b] + Dt[b * 3 + a]);
                }
            Rp.spd = (cholesky_ok(S6, 6) && cholesky_ok(S3k, 3) && cholesky_ok(S3d, 3)) ? 1 : 0;
            const double *Gm = &gm[(size_t)i * 36], *Gk = &gs[(size_t)i * 9], *Gd = &gs[(size_t)(batch + i) * 9];
            Rp.hill_mandel_gap = std::max(fro_ratio(Gm, Cm, 36), std::max(fro_ratio(Gk, Kt, 9), fro_ratio(Gd, Dt, 9)));
        }
        if (Rp.status != CHOM_OK) overall = CHOM_ENOCONV;
        if (rep) rep[i] = Rp;
    }
    if (dev) {
        CHOM_HIP(hipMemcpyAsync(C_hom, oc.data(), sizeof(double) * oc.size(), hipMemcpyHostToDevice, s));
        CHOM_HIP(hipMemcpyAsync(K_hom, ok.data(), sizeof(double) * ok.size(), hipMemcpyHostToDevice, s));
        CHOM_HIP(hipMemcpyAsync(D_hom, od.data(), sizeof(double) * od.size(), hipMemcpyHostToDevice, s));
        CHOM_HIP(hipStreamSynchronize(s));
    } else {
        std::memcpy(C_hom, oc.data(), sizeof(double) * oc.size());
        std::memcpy(K_hom, ok.data(), sizeof(double) * ok.size());
        std::memcpy(D_hom, od.data(), sizeof(double) * od.size());
    }
    if (overall != CHOM_OK) set_error("some load case did not converge");
    return overall;
}

static int check_options(const chom_options &o) {
    if (o.precision != CHOM_FP64 && o.precision != CHOM_FP32_REFINED) {
        set_error("unknown precision");
        return CHOM_EINVAL;
    }
    if (o.precond != CHOM_PRECOND_BLOCK_JACOBI && o.precond != CHOM_PRECOND_TWO_LEVEL) {
        set_error("unknown preconditioner");
        return CHOM_EINVAL;
    }
    if (!(o.rtol > 0) || !(o.inner_rtol > 0) || o.max_iter < 1 || o.max_refine < 0 || !(o.c_sat > 0)) {
        set_error("bad tolerances or caps");
        return CHOM_EINVAL;
    }
    return CHOM_OK;
}

static int64_t kuhn_vertex(int i, int j, int k, int n) { return i + (int64_t)(n + 1) * (j + (int64_t)(n + 1) * k); }

static int batch_time_operator(chom_batch *B, int32_t physics, int32_t reps, double *ms_per_launch,
                               int64_t *tets_per_launch, int32_t *problems_per_launch) {
    if (!B || !ms_per_launch || reps < 1 || (physics != 0 && physics != 1)) {
        set_error("time_operator: bad argument");
        return CHOM_EINVAL;
    }
    const bool f32 = B->opt.precision == CHOM_FP32_REFINED;
    if ((physics == 0 ? B->mech.L.nprob : B->scal.L.nprob) == 0) {
        set_error("time_operator: call the homogenise function first (the timing reuses its workspace)");
        return CHOM_EINVAL;
    }
    if (physics == 0) {
        if (f32) CHOM_TRY((time_op<float, 3, 6>(B, B->mech, B->mech.pf.p, B->mech.qf.p, B->mech.L.rg, reps, ms_per_launch)));
        else CHOM_TRY((time_op<double, 3, 6>(B, B->mech, B->mech.pd.p, B->mech.qd.p, B->mech.L.rg, reps, ms_per_launch)));
    } else {
        if (f32) CHOM_TRY((time_op<float, 1, 3>(B, B->scal, B->scal.pf.p, B->scal.qf.p, B->scal.L.rg, reps, ms_per_launch)));
        else CHOM_TRY((time_op<double, 1, 3>(B, B->scal, B->scal.pd.p, B->scal.qd.p, B->scal.L.rg, reps, ms_per_launch)));
    }
    int64_t tets = 0;
    for (auto *r : B->entries) tets += 6LL * r->n * r->n * r->n;
    if (tets_per_launch) *tets_per_launch = physics == 0 ? tets : 2 * tets;
    if (problems_per_launch) *problems_per_launch = physics == 0 ? (int)B->entries.size() : 2 * (int)B->entries.size();
    return CHOM_OK;
}

}  // namespace chom

// ====================================================================== C ABI
namespace chom {

int rve_homogenise_host(chom_rve *rve, const chom_params *params, int batch, double *C, double *K, double *D,
                        chom_report *rep) {
    if (!rve->self || rve->self_size != batch) {
        rve->self.reset();
        std::unique_ptr<chom_batch> B(new chom_batch());
        std::vector<chom_rve *> ents(batch, rve);
        CHOM_TRY(batch_init(B.get(), ents.data(), batch, &rve->opt));
        rve->self = std::move(B);
        rve->self_size = batch;
    }
    return batch_homogenise(rve->self.get(), params, C, K, D, rep, false);
}

void rve_settings(const chom_rve *rve, double *c_sat, int *degrade_yarn) {
    *c_sat = rve->opt.c_sat;
    *degrade_yarn = rve->opt.degrade_yarn;
}

}  // namespace chom

extern "C" {

const char *chom_last_error(void) { return chom::g_last_error.c_str(); }
const char *chom_version(void) { return "chom 0.2 (gfx950, order-2 lattice operator, batched)"; }

int chom_default_options(chom_options *opt) {
    if (!opt) return CHOM_EINVAL;
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = CHOM_FP64;
    opt->precond = CHOM_PRECOND_TWO_LEVEL;
    opt->max_iter = 20000;
    opt->max_refine = 30;
    opt->rtol = 1e-12;
    opt->inner_rtol = 1e-4;
    opt->c_sat = 1.5;
    return CHOM_OK;
}

int chom_mesh_sizes(int32_t n, int32_t *nv, int32_t *nt) {
    if (n < 1 || n > 1024 || !nv || !nt) {
        set_error("chom_mesh_sizes: n must be in [1, 1024] and outputs non-null");
        return CHOM_EINVAL;
    }
    const int64_t v = (int64_t)(n + 1) * (n + 1) * (n + 1), t = 6LL * n * n * n;
    if (t > INT32_MAX) {
        set_error("chom_mesh_sizes: mesh too large for 32-bit tet counts");
        return CHOM_EINVAL;
    }
    *nv = (int32_t)v;
    *nt = (int32_t)t;
    return CHOM_OK;
}

int chom_generate_plain_weave(int32_t n, double *coords, int32_t *tets, int8_t *phase, double *axis, void *stream) {
    int32_t nv, nt;
    int st = chom_mesh_sizes(n, &nv, &nt);
    if (st != CHOM_OK) return st;
    if (!coords || !tets || !phase || !axis) {
        set_error("chom_generate_plain_weave: null output buffer");
        return CHOM_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    CHOM_HIP(launch_generate(n, coords, tets, phase, axis, s));
    CHOM_HIP(hipStreamSynchronize(s));
    return CHOM_OK;
}

int chom_material_constants(const chom_materials *mat, const chom_params *params, double c_sat, int32_t degrade_yarn,
                            double *out_mech, double *out_therm, double *out_moist, double *omega_keep) {
    if (!mat || !out_mech || !out_therm || !out_moist) {
        set_error("chom_material_constants: null argument");
        return CHOM_EINVAL;
    }
    return material_constants(mat, params, c_sat, degrade_yarn, out_mech, out_therm, out_moist, omega_keep);
}

int chom_rve_create(const chom_mesh *mesh, const chom_materials *mat, int32_t bc, int32_t order,
                    const chom_options *opt, chom_rve **out) {
    if (!mesh || !mat || !out) {
        set_error("chom_rve_create: null argument");
        return CHOM_EINVAL;
    }
    *out = nullptr;
    if (bc < 0 || bc > 2) {
        set_error("chom_rve_create: bc_type must be 0 (Dirichlet), 1 (periodic) or 2 (Neumann)");
        return CHOM_EINVAL;
    }
    if (order < 2 || order > 4) {
        set_error("chom_rve_create: order must be 2, 3 or 4");
        return CHOM_EINVAL;
    }
    chom_options o;
    chom_default_options(&o);
    if (opt) o = *opt;
    {
        const int st = check_options(o);
        if (st != CHOM_OK) {
            set_error("chom_rve_create: " + g_last_error);
            return st;
        }
    }
    int n = (int)std::lround(std::cbrt((double)mesh->n_tets / 6.0));
    if (n < 1 || 6LL * n * n * n != mesh->n_tets || (int64_t)(n + 1) * (n + 1) * (n + 1) != mesh->n_vertices) {
        set_error("chom_rve_create: mesh is not a Kuhn lattice (need (n+1)^3 vertices and 6 n^3 tets)");
        return CHOM_EMESH;
    }
    {
        const long long side = (long long)order * n + 1;   // lattice points are indexed in 32 bits
        if (side * side * side >= (1LL << 31)) {
            set_error("chom_rve_create: lattice of (order n + 1)^3 points too large (limit 2^31)");
            return CHOM_EINVAL;
        }
    }
    if (!mesh->coords || !mesh->tets || !mesh->phase || !mesh->fibre_axis) {
        set_error("chom_rve_create: null mesh array");
        return CHOM_EINVAL;
    }
    for (int d = 0; d < 3; ++d)
        if (!(mesh->hi[d] > mesh->lo[d])) {
            set_error("chom_rve_create: box must have hi > lo");
            return CHOM_EMESH;
        }
    const int64_t nv = mesh->n_vertices, nt = mesh->n_tets;
    std::vector<double> hc(3 * nv), hax(3 * nt);
    std::vector<int32_t> ht(4 * nt);
    std::vector<int8_t> hph(nt);
    if (mesh->on_device) {
        CHOM_HIP(hipMemcpy(hc.data(), mesh->coords, sizeof(double) * 3 * nv, hipMemcpyDeviceToHost));
        CHOM_HIP(hipMemcpy(ht.data(), mesh->tets, sizeof(int32_t) * 4 * nt, hipMemcpyDeviceToHost));
        CHOM_HIP(hipMemcpy(hph.data(), mesh->phase, nt, hipMemcpyDeviceToHost));
        CHOM_HIP(hipMemcpy(hax.data(), mesh->fibre_axis, sizeof(double) * 3 * nt, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(hc.data(), mesh->coords, sizeof(double) * 3 * nv);
        std::memcpy(ht.data(), mesh->tets, sizeof(int32_t) * 4 * nt);
        std::memcpy(hph.data(), mesh->phase, nt);
        std::memcpy(hax.data(), mesh->fibre_axis, sizeof(double) * 3 * nt);
    }
    for (int64_t e = 0; e < nt; ++e) {
        const int t = (int)(e % 6);
        const int64_t cell = e / 6;
        const int ci = (int)(cell % n), cj = (int)((cell / n) % n), ck = (int)(cell / ((int64_t)n * n));
        int p0, p1;
        kuhn_perm(t, p0, p1);
        int v[4][3] = {{ci, cj, ck}, {ci, cj, ck}, {ci, cj, ck}, {ci + 1, cj + 1, ck + 1}};
        v[1][p0] += 1;
        v[2][p0] += 1;
        v[2][p1] += 1;
        int64_t want[4], got[4];
        for (int a = 0; a < 4; ++a) {
            want[a] = kuhn_vertex(v[a][0], v[a][1], v[a][2], n);
            got[a] = ht[4 * e + a];
        }
        std::sort(got, got + 4);
        for (int a = 0; a < 4; ++a)
            if (want[a] != got[a]) {
                set_error("chom_rve_create: tet " + std::to_string(e) + " does not match the Kuhn lattice");
                return CHOM_EMESH;
            }
        if (hph[e] < 0 || hph[e] > 4) {
            set_error("chom_rve_create: phase must be in 0..4");
            return CHOM_EMESH;
        }
        if (hph[e] > 0) {
            const double nr = std::sqrt(hax[3 * e] * hax[3 * e] + hax[3 * e + 1] * hax[3 * e + 1] + hax[3 * e + 2] * hax[3 * e + 2]);
            if (!(std::fabs(nr - 1.0) < 1e-6)) {
                set_error("chom_rve_create: yarn fibre axis must be a unit vector");
                return CHOM_EMESH;
            }
        }
    }
    bool uniform = true;
    double h[3];
    for (int d = 0; d < 3; ++d) h[d] = (mesh->hi[d] - mesh->lo[d]) / n;
    const double scale = std::max(mesh->hi[0] - mesh->lo[0], std::max(mesh->hi[1] - mesh->lo[1], mesh->hi[2] - mesh->lo[2]));
    const double tol = 1e-12 * scale;
    for (int k = 0; k <= n; ++k)
        for (int j = 0; j <= n; ++j)
            for (int i = 0; i <= n; ++i) {
                const int64_t v = kuhn_vertex(i, j, k, n);
                const int ijk[3] = {i, j, k};
                for (int d = 0; d < 3; ++d) {
                    const double ref = (ijk[d] == n) ? mesh->hi[d] : mesh->lo[d] + (mesh->hi[d] - mesh->lo[d]) * ((double)ijk[d] / n);
                    const double x = hc[3 * v + d];
                    if (std::fabs(x - ref) > tol) uniform = false;
                    if ((ijk[d] == 0 && std::fabs(x - mesh->lo[d]) > tol) || (ijk[d] == n && std::fabs(x - mesh->hi[d]) > tol)) {
                        set_error("chom_rve_create: boundary vertex off its face");
                        return CHOM_EMESH;
                    }
                }
                if (bc == CHOM_BC_PERIODIC) {
                    for (int d = 0; d < 3; ++d) {
                        if (ijk[d] != n) continue;
                        int m[3] = {i, j, k};
                        m[d] = 0;
                        const int64_t w = kuhn_vertex(m[0], m[1], m[2], n);
                        for (int d2 = 0; d2 < 3; ++d2)
                            if (d2 != d && std::fabs(hc[3 * v + d2] - hc[3 * w + d2]) > tol) {
                                set_error("chom_rve_create: periodic faces do not match");
                                return CHOM_EMESH;
                            }
                    }
                }
            }
    {
        double m10[10], t4[4], d4[4];
        if (material_constants(mat, nullptr, o.c_sat, o.degrade_yarn, m10, t4, d4, nullptr) != CHOM_OK) return CHOM_EMATERIAL;
    }
    std::unique_ptr<chom_rve> R(new chom_rve());
    R->n = n;
    R->bc = bc;
    R->order = order;
    for (int d = 0; d < 3; ++d) {
        R->lo[d] = mesh->lo[d];
        R->hi[d] = mesh->hi[d];
    }
    R->mat = *mat;
    R->opt = o;
    Geo &G = R->geo;
    std::memset(&G, 0, sizeof(G));
    G.n = n;
    G.bc = bc;
    G.uniform = uniform ? 1 : 0;
    G.p = order;
    G.L = order * n;
    G.Lw = (bc == CHOM_BC_PERIODIC) ? G.L : G.L + 1;
    G.npts = (long long)G.Lw * G.Lw * G.Lw;
    G.volume = (mesh->hi[0] - mesh->lo[0]) * (mesh->hi[1] - mesh->lo[1]) * (mesh->hi[2] - mesh->lo[2]);
    G.nrow = (bc == CHOM_BC_DIRICHLET) ? 0 : (bc == CHOM_BC_PERIODIC ? 1 : 4);
    G.tiles_x = (n + TX - 1) / TX;
    G.tiles_y = (n + TY - 1) / TY;
    G.tiles_z = (n + TZ - 1) / TZ;
    G.ntiles = G.tiles_x * G.tiles_y * G.tiles_z;
    G.tcx = TX;
    G.tcy = TY;
    G.tcz = TZ;
    if (order != 2) {   // orders 3, 4: one cell per operator tile
        G.tiles_x = G.tiles_y = G.tiles_z = n;
        G.ntiles = n * n * n;
        G.tcx = G.tcy = G.tcz = 1;
    }
    G.bx = order * G.tcx + 1;
    G.by = order * G.tcy + 1;
    G.bz = order * G.tcz + 1;
    G.boxpts = G.bx * G.by * G.bz;
    mg_levels(G);
    for (int t = 0; t < 6; ++t) {
        int p0, p1;
        kuhn_perm(t, p0, p1);
        double v1[3] = {0, 0, 0}, v2[3] = {0, 0, 0}, v3[3] = {h[0], h[1], h[2]};
        v1[p0] = h[p0];
        v2[p0] = h[p0];
        v2[p1] = h[p1];
        const double J[3][3] = {{v1[0], v2[0], v3[0]}, {v1[1], v2[1], v3[1]}, {v1[2], v2[2], v3[2]}};
        const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        const double id = 1.0 / det;
        const double Ji[3][3] = {
            {(J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id, (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id, (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id},
            {(J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id, (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id, (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id},
            {(J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id, (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id, (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id}};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                G.tg64[t][3 * i + j] = Ji[i][j];
                G.tg32[t][3 * i + j] = (float)Ji[i][j];
            }
        G.tg64[t][9] = std::fabs(det) / 6.0;
        G.tg32[t][9] = (float)(std::fabs(det) / 6.0);
    }
    hipStream_t s = (hipStream_t)o.hip_stream;
    CHOM_HIP(R->elem64.ensure(nt));
    CHOM_HIP(R->elem32.ensure(nt));
    if (!uniform) {
        CHOM_HIP(R->geo64.ensure(10 * nt));
        CHOM_HIP(R->geo32.ensure(10 * nt));
    }
    CHOM_HIP(R->rows.ensure(4 * G.npts));
    DevBuf<double> dc, dax;
    DevBuf<int8_t> dph;
    DevBuf<int> dbad;
    CHOM_HIP(dc.ensure(3 * nv));
    CHOM_HIP(dax.ensure(3 * nt));
    CHOM_HIP(dph.ensure(nt));
    CHOM_HIP(dbad.ensure(1));
    CHOM_HIP(hipMemcpyAsync(dc.p, hc.data(), sizeof(double) * 3 * nv, hipMemcpyHostToDevice, s));
    CHOM_HIP(hipMemcpyAsync(dax.p, hax.data(), sizeof(double) * 3 * nt, hipMemcpyHostToDevice, s));
    CHOM_HIP(hipMemcpyAsync(dph.p, hph.data(), nt, hipMemcpyHostToDevice, s));
    CHOM_HIP(hipMemsetAsync(dbad.p, 0, sizeof(int), s));
    G.elem64 = R->elem64.p;
    G.elem32 = R->elem32.p;
    G.geo64 = uniform ? nullptr : R->geo64.p;
    G.geo32 = uniform ? nullptr : R->geo32.p;
    G.rows = R->rows.p;
    if (G.mg_nlev > 0) {
        std::vector<int> nb, ch, pa;
        mg_tables(G, nb, ch, pa);
        CHOM_HIP(R->mg_nbr.ensure(nb.size()));
        CHOM_HIP(R->mg_child.ensure(ch.size()));
        CHOM_HIP(R->mg_par.ensure(pa.size()));
        CHOM_HIP(hipMemcpy(R->mg_nbr.p, nb.data(), sizeof(int) * nb.size(), hipMemcpyHostToDevice));
        CHOM_HIP(hipMemcpy(R->mg_child.p, ch.data(), sizeof(int) * ch.size(), hipMemcpyHostToDevice));
        CHOM_HIP(hipMemcpy(R->mg_par.p, pa.data(), sizeof(int) * pa.size(), hipMemcpyHostToDevice));
        G.mg_nbr = R->mg_nbr.p;
        G.mg_child = R->mg_child.p;
        G.mg_par = R->mg_par.p;
    }
    if (order != 2) {
        hp::HostTables tb;
        if (!hp::build_tables(order, tb)) {
            set_error("chom_rve_create: order-" + std::to_string(order) + " tables failed");
            return CHOM_EINVAL;
        }
        const int ne = tb.ne, m3 = 3 * tb.m;
        int MA, KA, MB, KB;
        if (order == 3) {
            MA = hp::Shape<3>::MA; KA = hp::Shape<3>::KA; MB = hp::Shape<3>::MB; KB = hp::Shape<3>::KB;
        } else {
            MA = hp::Shape<4>::MA; KA = hp::Shape<4>::KA; MB = hp::Shape<4>::MB; KB = hp::Shape<4>::KB;
        }
        std::vector<double> DA((size_t)MA * KA, 0.0), DB((size_t)MB * KB, 0.0);
        for (int r = 0; r < m3; ++r)
            for (int j = 0; j < ne; ++j) {
                DA[(size_t)r * KA + j] = tb.D[(size_t)r * ne + j];
                DB[(size_t)j * KB + r] = tb.D[(size_t)r * ne + j];
            }
        std::vector<float> DA32(DA.begin(), DA.end()), DB32(DB.begin(), DB.end());
        CHOM_HIP(R->hoff.ensure(tb.off.size()));
        CHOM_HIP(R->hW.ensure(tb.W.size()));
        CHOM_HIP(R->hWd.ensure(tb.Wd.size()));
        CHOM_HIP(R->hSd.ensure(tb.Sd.size()));
        CHOM_HIP(R->hDA64.ensure(DA.size()));
        CHOM_HIP(R->hDB64.ensure(DB.size()));
        CHOM_HIP(R->hDA32.ensure(DA.size()));
        CHOM_HIP(R->hDB32.ensure(DB.size()));
        CHOM_HIP(hipMemcpy(R->hoff.p, tb.off.data(), sizeof(int) * tb.off.size(), hipMemcpyHostToDevice));
        CHOM_HIP(hipMemcpy(R->hW.p, tb.W.data(), sizeof(double) * tb.W.size(), hipMemcpyHostToDevice));
        CHOM_HIP(hipMemcpy(R->hWd.p, tb.Wd.data(), sizeof(double) * tb.Wd.size(), hipMemcpyHostToDevice));
        CHOM_HIP(hipMemcpy(R->hSd.p, tb.Sd.data(), sizeof(double) * tb.Sd.size(), hipMemcpyHostToDevice));
        CHOM_HIP(hipMemcpy(R->hDA64.p, DA.data(), sizeof(double) * DA.size(), hipMemcpyHostToDevice));
        CHOM_HIP(hipMemcpy(R->hDB64.p, DB.data(), sizeof(double) * DB.size(), hipMemcpyHostToDevice));
        CHOM_HIP(hipMemcpy(R->hDA32.p, DA32.data(), sizeof(float) * DA32.size(), hipMemcpyHostToDevice));
        CHOM_HIP(hipMemcpy(R->hDB32.p, DB32.data(), sizeof(float) * DB32.size(), hipMemcpyHostToDevice));
        G.hoff = R->hoff.p;
        G.hW = R->hW.p;
        G.hWd = R->hWd.p;
        G.hSd = R->hSd.p;
        G.hDA64 = R->hDA64.p;
        G.hDB64 = R->hDB64.p;
        G.hDA32 = R->hDA32.p;
        G.hDB32 = R->hDB32.p;
    }
    CHOM_HIP(launch_element_setup(G, dc.p, nullptr, dph.p, dax.p, R->elem64.p, R->elem32.p, G.geo64 ? R->geo64.p : nullptr,
                                  G.geo32 ? R->geo32.p : nullptr, dbad.p, s));
    CHOM_HIP(launch_rows(G, R->rows.p, s));
    int hbad = 0;
    CHOM_HIP(hipMemcpyAsync(&hbad, dbad.p, sizeof(int), hipMemcpyDeviceToHost, s));
    CHOM_HIP(hipStreamSynchronize(s));
    if (hbad) {
        set_error("chom_rve_create: " + std::to_string(hbad) + " tets are degenerate or inverted");
        return CHOM_EMESH;
    }
    *out = R.release();
    return CHOM_OK;
}

void chom_rve_destroy(chom_rve *rve) { delete rve; }

int chom_homogenise(chom_rve *rve, const chom_params *params, int32_t batch, double *C_hom, double *K_hom,
                    double *D_hom, chom_report *rep) {
    if (!rve || !params || !C_hom || !K_hom || !D_hom || batch < 1) {
        set_error("chom_homogenise: null argument or batch < 1");
        return CHOM_EINVAL;
    }
    if (!rve->self || rve->self_size != batch) {
        rve->self.reset();
        std::unique_ptr<chom_batch> B(new chom_batch());
        std::vector<chom_rve *> ents(batch, rve);
        const int st = batch_init(B.get(), ents.data(), batch, &rve->opt);
        if (st != CHOM_OK) return st;
        rve->self = std::move(B);
        rve->self_size = batch;
    }
    const int st = batch_homogenise(rve->self.get(), params, C_hom, K_hom, D_hom, rep, rve->opt.device_ptrs != 0);
    if (st != CHOM_OK) set_error("chom_homogenise: " + g_last_error);
    return st;
}

int chom_time_operator(chom_rve *rve, int32_t physics, int32_t reps, double *ms_per_launch, int64_t *tets_per_launch,
                       int32_t *problems_per_launch) {
    if (!rve || !rve->self) {
        set_error("chom_time_operator: call chom_homogenise first (the timing reuses its workspace)");
        return CHOM_EINVAL;
    }
    return batch_time_operator(rve->self.get(), physics, reps, ms_per_launch, tets_per_launch, problems_per_launch);
}

int chom_batch_create(chom_rve *const *rves, int32_t n, const chom_options *opt, chom_batch **out) {
    if (!rves || n < 1 || !out) {
        set_error("chom_batch_create: null argument or n < 1");
        return CHOM_EINVAL;
    }
    *out = nullptr;
    for (int i = 0; i < n; ++i)
        if (!rves[i]) {
            set_error("chom_batch_create: null RVE handle");
            return CHOM_EINVAL;
        }
    chom_options o = rves[0]->opt;
    if (opt) o = *opt;
    CHOM_TRY(check_options(o));
    std::unique_ptr<chom_batch> B(new chom_batch());
    CHOM_TRY(batch_init(B.get(), rves, n, &o));
    *out = B.release();
    return CHOM_OK;
}

int chom_batch_homogenise(chom_batch *batch, const chom_params *params, double *C_hom, double *K_hom, double *D_hom,
                          chom_report *rep) {
    if (!batch || !params || !C_hom || !K_hom || !D_hom) {
        set_error("chom_batch_homogenise: null argument");
        return CHOM_EINVAL;
    }
    const int st = batch_homogenise(batch, params, C_hom, K_hom, D_hom, rep, batch->opt.device_ptrs != 0);
    if (st != CHOM_OK) set_error("chom_batch_homogenise: " + g_last_error);
    return st;
}

int chom_batch_time_operator(chom_batch *batch, int32_t physics, int32_t reps, double *ms_per_launch,
                             int64_t *tets_per_launch, int32_t *problems_per_launch) {
    return batch_time_operator(batch, physics, reps, ms_per_launch, tets_per_launch, problems_per_launch);
}

int chom_batch_launch_config(const chom_batch *batch, int32_t *rg_mech, int32_t *rg_scal, int32_t *nwg_mech,
                             int32_t *nwg_scal) {
    if (!batch) {
        set_error("chom_batch_launch_config: null batch");
        return CHOM_EINVAL;
    }
    if (rg_mech) *rg_mech = batch->rg_mech;
    if (rg_scal) *rg_scal = batch->rg_scal;
    if (nwg_mech) *nwg_mech = batch->mech.L.nwg;
    if (nwg_scal) *nwg_scal = batch->scal.L.nwg;
    return CHOM_OK;
}

void chom_batch_destroy(chom_batch *batch) { delete batch; }

int chom_element_apply_host(int32_t ncomp, const double *grad_lam, double vol, const double *axis, const double *inv5,
                            const double *u, double *y) {
    if (!grad_lam || !axis || !inv5 || !u || !y || (ncomp != 1 && ncomp != 3)) {
        set_error("chom_element_apply_host: bad argument");
        return CHOM_EINVAL;
    }
    double g[4][3], a[3] = {axis[0], axis[1], axis[2]}, m[5];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 3; ++j) g[i][j] = grad_lam[3 * i + j];
    for (int k = 0; k < 5; ++k) m[k] = inv5[k];
    if (ncomp == 3) {
        double uu[10][3], yy[10][3];
        for (int k = 0; k < 10; ++k)
            for (int c = 0; c < 3; ++c) uu[k][c] = u[3 * k + c];
        p2_apply<double, 3>(g, vol, a, m, uu, yy);
        for (int k = 0; k < 10; ++k)
            for (int c = 0; c < 3; ++c) y[3 * k + c] = yy[k][c];
    } else {
        double uu[10][1], yy[10][1];
        for (int k = 0; k < 10; ++k) uu[k][0] = u[k];
        p2_apply<double, 1>(g, vol, a, m, uu, yy);
        for (int k = 0; k < 10; ++k) y[k] = yy[k][0];
    }
    return CHOM_OK;
}

int chom_basis_tables_host(int32_t order, int32_t *n_e, int32_t *m, double *S, double *W, double *Wd,
                           int32_t *offsets) {
    chom::hp::HostTables t;
    if (!chom::hp::build_tables(order, t)) {
        set_error("chom_basis_tables_host: order must be 3 or 4");
        return CHOM_EINVAL;
    }
    if (n_e) *n_e = t.ne;
    if (m) *m = t.m;
    if (S) std::copy(t.S.begin(), t.S.end(), S);
    if (W) std::copy(t.W.begin(), t.W.end(), W);
    if (Wd) std::copy(t.Wd.begin(), t.Wd.end(), Wd);
    if (offsets) std::copy(t.off.begin(), t.off.end(), offsets);
    return CHOM_OK;
}

int chom_basis_eval_host(int32_t order, const double *lam, double *out) {
    if (!lam || !out || !chom::hp::eval_basis(order, lam, out)) {
        set_error("chom_basis_eval_host: order must be 3 or 4 and pointers non-null");
        return CHOM_EINVAL;
    }
    return CHOM_OK;
}

}  // extern "C"
