// Preconditioned conjugate gradients on the constrained RVE system, many
// problems (parameter records x RVEs, possibly of different sizes and BCs) and
// load cases at once.
//
// The paper solves the saddle-point system of Eq. eq_RVE_disc_Eqs with a
// direct factorisation; it notes that projection is an equivalent route (Sec.
// 2, after Eq. eq_X_mech).  Here the fluctuation is found by CG on ker(C): with
// the block-Jacobi preconditioner M and the constraint rows C (periodic: the
// mean of each component; uniform traction: the surface moments and the mean),
// the preconditioner is z = P M^-1 r with the M-oblique projector
//   P M^-1 = M^-1 - M^-1 C^T (C M^-1 C^T)^-1 C M^-1,
// which maps into ker(C) and annihilates range(C^T).  The residual is
// re-projected with the adjoint projector every iteration, so the multiplier
// forces do not accumulate in r and r.z stays accurate.  r.z, its pieces and
// p.Kp are accumulated in FP64 whatever the vector precision.
//
// Vectors are load-case major: [problem][load case][point][component].
// Vector kernels: a workgroup is R waves; wave w handles load case w of 64
// consecutive lattice points at a time (contiguous accesses; grid-stride over
// the problem's point blocks) and reduces its own column, so partial sums
// need no block barrier.
// Partial layout (k-major): partial[((prob * R + w) * REC + k) * nwg + block],
// REC = 2 + C * NR with NR the largest row count of the launch; record
// [r.z0, r.r, C z0 (C x NR, entry c * NR + a)].
#include "common.h"
#include "internal.h"

namespace chom {

// Partial record of this wave: slot `slot` of `stride` slots per entry.
template <int REC>
__device__ inline void wave_partials(double *acc, double *partial, int prob, int R, int w, int stride, int slot) {
    const int lane = threadIdx.x & 63;
    int k;
    const double s = wave_sums_spread<REC>(acc, k);
    if (wave_spread_writer<REC>(lane) && k < REC) partial[(((long long)prob * R + w) * REC + k) * stride + slot] = s;
}
template <int REC>
__device__ inline void wave_partials(double *acc, double *partial, int prob, int R, int w) {
    wave_partials<REC>(acc, partial, prob, R, w, gridDim.x, blockIdx.x);
}

// Adds this wave's record to the striped accumulators of its column (see ACC_STRIPES).
template <int C, int REC>
__device__ inline void wave_accum(double *acc, double *accbuf, int prob, int R, int w) {
    const int lane = threadIdx.x & 63;
    const int stripe = blockIdx.x & (ACC_STRIPES - 1);
    int k;
    const double s = wave_sums_spread<REC>(acc, k);
    if (wave_spread_writer<REC>(lane) && k < REC) unsafeAtomicAdd(&accbuf[acc_index<C>(prob, R, w, k, stripe)], s);
}

// r = b, x = 0; partial sums of r, z0 = M^-1 r.  WRITE = false: only the sums.
template <typename T, int C, int R, int NR, bool WRITE>
__global__ __launch_bounds__(64 * R) void cg_init_kernel(const Geo *__restrict__ geos, const Prob *__restrict__ probs, const T *b, T *x,
                                                         T *r, const T *minv, double *accbuf) {
    constexpr int MS = (C == 3) ? 6 : 1;
    constexpr int REC = 2 + C * NR;
    const int prob = blockIdx.y;
    const Prob &P = probs[prob];
    const Geo &G = geos[P.geo];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const T *Mp = minv + P.doff * MS;
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
        double row[4];
        load_rows<NR>(G, pt, row);
        const long long o = P.voff + (w * G.npts + pt) * C;
        T rv[C], zv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) rv[c] = b[o + c];
        minv_apply<T, C>(Mi, rv, zv);
        if constexpr (WRITE) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                r[o + c] = rv[c];
                x[o + c] = T(0);
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
    wave_accum<C, REC>(acc, accbuf, prob, R, w);
}

// x += alpha p (the step length of the previous iteration, applied here while
// p is read anyway; cg_flush_x_kernel applies the last one) ; z = z0 - M^-1 C^T y ;
// r = r - C^T y ; p = z + beta p.  With the two-level
// preconditioner (mg.on) the vertex points also take the coarse correction
// z += Q f, f = e1 - W y on the n/2 grid (e1 = V Q^T r, W = V Q^T C^T, formed by
// mg_fcorr_kernel), Q = P_0 P_1 (P_0 injects vertex values, P_1 interpolates
// from the n/2 grid).
//
// Wave g takes load cases KG g .. KG g + KG - 1, so a point's inverse block,
// constraint rows and coarse-grid parents are found once for all of them.
template <typename T, int C, int R, int NR, int KG>
__global__ __launch_bounds__(64 * (R / KG)) void cg_dir_kernel(const Geo *__restrict__ geos,
                                                               const Prob *__restrict__ probs, T *x, T *r, T *p,
                                                               const T *minv, const double *ycoef,
                                                               const ColState *cols, const int *prob_active,
                                                               MgDir<T> mg) {
    constexpr int MS = (C == 3) ? 6 : 1;
    constexpr int S = C * NR;
    const int prob = blockIdx.y;
    const int g = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c0 = g * KG;
    // a finished problem still takes the pending x update of its last step
    // (the finishing kernel zeroes alpha of finished columns afterwards)
    const bool active = prob_active[prob] != 0;
    double alpha[KG], beta[KG];
    bool any_alpha = false, any_move = false;
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) {
        alpha[kk] = cols[prob * R + c0 + kk].alpha;
        beta[kk] = cols[prob * R + c0 + kk].beta;
        any_alpha = any_alpha || alpha[kk] != 0.0;
        any_move = any_move || alpha[kk] != 0.0 || beta[kk] != 0.0;
    }
    if (!active && !any_alpha) return;   // per wave: the kernel has no block barrier
    const Prob &P = probs[prob];
    const Geo &G = geos[P.geo];
    double yv[KG][S > 0 ? S : 1];
#pragma unroll
    for (int kk = 0; kk < KG; ++kk)
#pragma unroll
        for (int k = 0; k < S; ++k) yv[kk][k] = ycoef[((long long)prob * R + c0 + kk) * S + k];
    const T *Mp = minv + P.doff * MS;
    const bool proj = (NR > 0) && G.nrow > 0;
    const long long nblk = (G.npts + 63) / 64;
    for (long long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const long long pt = blk * 64 + lane;
        if (pt >= G.npts) continue;
        // every load that does not depend on another is issued before any use
        // (alpha, beta and active are uniform over the wave)
        T pv[KG][C], xv[KG][C], rv[KG][C], Mi[MS];
        double row[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
            const long long o = P.voff + ((c0 + kk) * G.npts + pt) * C;
            if (any_move) {
#pragma unroll
                for (int c = 0; c < C; ++c) pv[kk][c] = p[o + c];
            }
            if (any_alpha) {
#pragma unroll
                for (int c = 0; c < C; ++c) xv[kk][c] = x[o + c];
            }
            if (active) {
#pragma unroll
                for (int c = 0; c < C; ++c) rv[kk][c] = r[o + c];
            }
        }
        long long J0 = -1, J1 = -1;
        if (active) {
#pragma unroll
            for (int k = 0; k < MS; ++k) Mi[k] = Mp[pt * MS + k];
            if (proj) load_rows<NR>(G, pt, row);
            if (mg.on && G.mg_nlev > 0) {
                int X, Y, Z;
                lattice_xyz(G, pt, X, Y, Z);
                const int pp = G.p;
                if (X % pp == 0 && Y % pp == 0 && Z % pp == 0) {
                    // vertex (i, j, k): f at its level-1 parents (itself halved, or the two
                    // ends of the level-1 Kuhn edge whose midpoint it is), averaged
                    const int lw0 = G.mg_lw[0];
                    const long long v = X / pp + (long long)lw0 * (Y / pp + (long long)lw0 * (Z / pp));
                    const int *pa = G.mg_par + (G.mg_off[0] + v) * 16;
                    J0 = pa[0];
                    J1 = pa[1];
                }
            }
        }
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
            const long long o = P.voff + ((c0 + kk) * G.npts + pt) * C;
            if (alpha[kk] != 0.0) {
                const T al = (T)alpha[kk];
#pragma unroll
                for (int c = 0; c < C; ++c) x[o + c] = xv[kk][c] + al * pv[kk][c];
            }
            if (!active) continue;
            T zv[C];
            minv_apply<T, C>(Mi, rv[kk], zv);   // z0 = M^-1 r, as in the update kernel's sums
            if constexpr (NR > 0) {
                if (proj) {
                    // projection correction M^-1 C^T y evaluated in FP64
                    double Md[MS], ct[C], corr[C];
#pragma unroll
                    for (int k = 0; k < MS; ++k) Md[k] = (double)Mi[k];
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        ct[c] = 0.0;
#pragma unroll
                        for (int a = 0; a < NR; ++a) ct[c] += row[a] * yv[kk][c * NR + a];
                    }
                    minv_apply<double, C>(Md, ct, corr);
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        zv[c] = (T)((double)zv[c] - corr[c]);
                        r[o + c] = (T)((double)rv[kk][c] - ct[c]);
                    }
                }
            }
            if (J0 >= 0) {
                const T *f = mg.x0 + (P.moff * R + (long long)(c0 + kk) * G.mg_pts + G.mg_off[1]) * C;
#pragma unroll
                for (int c = 0; c < C; ++c) zv[c] += T(0.5) * (f[J0 * C + c] + f[J1 * C + c]);
            }
            if (beta[kk] == 0.0) {   // first step (p not yet defined) or finished column
#pragma unroll
                for (int c = 0; c < C; ++c) p[o + c] = zv[c];
            } else {
                const T bt = (T)beta[kk];
#pragma unroll
                for (int c = 0; c < C; ++c) p[o + c] = zv[c] + bt * pv[kk][c];
            }
        }
    }
}

// Sum of the tile-box copies of lattice point (X, Y, Z) for load cases c0 ..
// c0 + KG - 1, which lie in one operator group (boxes [tile][group][case in
// group][box point][C], rg cases per group, ng groups), in the vector precision.
// Every copy of every case is loaded before any is summed.
template <typename T, int C, int KG>
__device__ inline void gather_tiles_grp(const Geo &G, const T *qt, int ng, int rg, int c0, int X, int Y, int Z,
                                        T out[KG][C]) {
    const int grp = c0 / rg, rr0 = c0 - grp * rg;
    const bool per = (G.bc == 1);
    const int m2 = G.L;
    int tx[2], ty[2], tz[2], lx[2], ly[2], lz[2];
    const int nx = tile_cands(X, G.p * G.tcx, G.tiles_x, m2, per, tx, lx);
    const int ny = tile_cands(Y, G.p * G.tcy, G.tiles_y, m2, per, ty, ly);
    const int nz = tile_cands(Z, G.p * G.tcz, G.tiles_z, m2, per, tz, lz);
    T cp[8][KG][C];
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int kk = 0; kk < KG; ++kk)
#pragma unroll
            for (int v = 0; v < C; ++v) cp[k][kk][v] = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (a < nx && b < ny && c < nz) {
                    // 32-bit: one problem's tile boxes hold fewer than 2^31 values (checked at setup)
                    const int tile = tx[a] + G.tiles_x * (ty[b] + G.tiles_y * tz[c]);
                    const int off = (((tile * ng + grp) * rg + rr0) * G.boxpts + lx[a] + G.bx * (ly[b] + G.by * lz[c])) * C;
#pragma unroll
                    for (int kk = 0; kk < KG; ++kk)
#pragma unroll
                        for (int v = 0; v < C; ++v) cp[4 * a + 2 * b + c][kk][v] = qt[off + kk * G.boxpts * C + v];
                }
            }
#pragma unroll
    for (int kk = 0; kk < KG; ++kk)
#pragma unroll
        for (int v = 0; v < C; ++v) {
            T sum = T(0);
#pragma unroll
            for (int k = 0; k < 8; ++k) sum += cp[k][kk][v];
            out[kk][v] = sum;
        }
}

// r -= alpha q (q gathered from the operator's tile boxes) ; partial sums of r
// and z0 = M^-1 r (z0 itself is formed again by the direction kernel, which
// reads r anyway; x += alpha p is deferred to the next direction kernel).
// Wave g takes load cases KG g .. KG g + KG - 1 (KG divides the operator's
// load cases per group, rg), so a point's lattice position, tile-box addresses,
// inverse block and constraint rows are found once for all of them.
template <typename T, int C, int R, int NR, int KG>
__global__ __launch_bounds__(64 * (R / KG)) void cg_update_kernel(const Geo *__restrict__ geos,
                                                                  const Prob *__restrict__ probs, int rg, T *r,
                                                                  const T *q, const T *minv, const ColState *cols,
                                                                  double *accbuf, const int *prob_active) {
    constexpr int MS = (C == 3) ? 6 : 1;
    constexpr int REC = 2 + C * NR;
    const int prob = blockIdx.y;
    const int grp = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double acc[KG][REC];
#pragma unroll
    for (int kk = 0; kk < KG; ++kk)
#pragma unroll
        for (int k = 0; k < REC; ++k) acc[kk][k] = 0.0;
    if (prob_active[prob] == 0) return;
    const Prob &P = probs[prob];
    const Geo &G = geos[P.geo];
    T al[KG];
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) al[kk] = (T)cols[prob * R + grp * KG + kk].alpha;
    const T *Mp = minv + P.doff * MS;
    const T *qt = q + P.qoff;
    const long long nblk = (G.npts + 63) / 64;
    for (long long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const long long pt = blk * 64 + lane;
        if (pt >= G.npts) continue;
        // the point's own loads first, then the gather: all in flight together
        T Mi[MS], rv[KG][C], qv[KG][C];
#pragma unroll
        for (int k = 0; k < MS; ++k) Mi[k] = Mp[pt * MS + k];
#pragma unroll
        for (int kk = 0; kk < KG; ++kk)
#pragma unroll
            for (int c = 0; c < C; ++c) rv[kk][c] = r[P.voff + ((grp * KG + kk) * G.npts + pt) * C + c];
        double row[4];
        load_rows<NR>(G, pt, row);
        int X, Y, Z;
        lattice_xyz(G, pt, X, Y, Z);
        if (dirichlet_boundary(G, X, Y, Z)) {
#pragma unroll
            for (int kk = 0; kk < KG; ++kk)
#pragma unroll
                for (int c = 0; c < C; ++c) qv[kk][c] = T(0);
        } else {
            gather_tiles_grp<T, C, KG>(G, qt, R / rg, rg, grp * KG, X, Y, Z, qv);
        }
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) {
            const long long o = P.voff + ((grp * KG + kk) * G.npts + pt) * C;
            T zv[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                rv[kk][c] = rv[kk][c] - al[kk] * qv[kk][c];
                r[o + c] = rv[kk][c];
            }
            minv_apply<T, C>(Mi, rv[kk], zv);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                acc[kk][0] += (double)rv[kk][c] * (double)zv[c];
                acc[kk][1] += (double)rv[kk][c] * (double)rv[kk][c];
#pragma unroll
                for (int a = 0; a < NR; ++a) acc[kk][2 + c * NR + a] += row[a] * (double)zv[c];
            }
        }
    }
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) wave_accum<C, REC>(acc[kk], accbuf, prob, R, grp * KG + kk);
}

// x += alpha p with the pending step length of each column (after the last CG
// step of a solve).
template <typename T, int C, int R>
__global__ __launch_bounds__(64 * R) void cg_flush_x_kernel(const Geo *geos, const Prob *probs, T *x, const T *p,
                                                            const ColState *cols) {
    const int prob = blockIdx.y;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double alpha = cols[prob * R + w].alpha;
    if (alpha == 0.0) return;
    const Prob &P = probs[prob];
    const Geo &G = geos[P.geo];
    const T al = (T)alpha;
    const long long nblk = (G.npts + 63) / 64;
    for (long long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const long long pt = blk * 64 + lane;
        if (pt >= G.npts) continue;
        const long long o = P.voff + (w * G.npts + pt) * C;
#pragma unroll
        for (int c = 0; c < C; ++c) x[o + c] += al * p[o + c];
    }
}

// Outer (refinement) residual projected as a vector: r64 <- r64 - C^T y with
// y = (C M^-1 C^T)^-1 C M^-1 r64 from the previous reduction, r32 = (float) r64,
// and the partial sums of the projected residual.  Taking the norm of the
// projected vector keeps the multiplier forces of the exact solution out of
// the FP64 stopping test.
template <int C, int R, int NR>
__global__ __launch_bounds__(64 * R) void proj_resid_kernel(const Geo *__restrict__ geos, const Prob *__restrict__ probs, double *r64,
                                                            float *r32, const double *minv64,
                                                            const double *ycoef, double *accbuf) {
    constexpr int MS = (C == 3) ? 6 : 1;
    constexpr int REC = 2 + C * NR;
    constexpr int S = C * NR;
    const int prob = blockIdx.y;
    const Prob &P = probs[prob];
    const Geo &G = geos[P.geo];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double acc[REC];
#pragma unroll
    for (int k = 0; k < REC; ++k) acc[k] = 0.0;
    double yv[S > 0 ? S : 1];
#pragma unroll
    for (int k = 0; k < S; ++k) yv[k] = ycoef[((long long)prob * R + w) * S + k];
    const double *Mp = minv64 + P.doff * MS;
    const long long nblk = (G.npts + 63) / 64;
    for (long long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const long long pt = blk * 64 + lane;
        if (pt >= G.npts) continue;
        double Mi[MS];
#pragma unroll
        for (int k = 0; k < MS; ++k) Mi[k] = Mp[pt * MS + k];
        double row[4];
        load_rows<NR>(G, pt, row);
        const long long o = P.voff + (w * G.npts + pt) * C;
        double rv[C], zv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            double ct = 0.0;
#pragma unroll
            for (int a = 0; a < NR; ++a) ct += row[a] * yv[c * NR + a];
            rv[c] = r64[o + c] - ct;
            r64[o + c] = rv[c];
            if (r32) r32[o + c] = (float)rv[c];
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
    wave_accum<C, REC>(acc, accbuf, prob, R, w);
}

// Sum of part[k][0..nparts) for k in [0, K) into sums[k]; wave q takes
// k = q, q + nwaves, ...; coalesced loads, 4 independent chains per lane.
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

// alpha = r.z / p.Kp per column; p.Kp is read from the operator's striped
// accumulators ([prob][R][ACC_STRIPES]), which are cleared for the next step.
// One workgroup per problem.
template <int R>
__global__ __launch_bounds__(256) void finish_alpha_kernel(double *acc_pq, ColState *cols) {
    __shared__ double vals[R * ACC_STRIPES];
    const int prob = blockIdx.x;
    for (int t = threadIdx.x; t < R * ACC_STRIPES; t += blockDim.x) {
        double *a = acc_pq + (long long)prob * R * ACC_STRIPES + t;
        vals[t] = *a;
        *a = 0.0;
    }
    __syncthreads();
    if (threadIdx.x < R) {
        double v = 0.0;
        for (int st = 0; st < ACC_STRIPES; ++st) v += vals[threadIdx.x * ACC_STRIPES + st];
        ColState &cs = cols[prob * R + threadIdx.x];
        cs.pq = v;
        if (cs.done) {
            cs.alpha = 0.0;
        } else if (!isfinite(v)) {
            cs.alpha = 0.0;
            cs.done = COL_NONFINITE;
        } else if (!(v > 0.0)) {
            cs.alpha = 0.0;
            cs.done = COL_BREAKDOWN;
        } else {
            cs.alpha = cs.rz / v;
            // a CG step lowers the energy functional of the total field by alpha r.z
            cs.energy -= cs.alpha * cs.rz;
        }
    }
}

// rz = r.z0 - c^T (C M^-1 C^T)^-1 c, projection coefficients y, beta, convergence;
// the records [R][REC] are read from the vector kernels' striped accumulators,
// which are cleared for the next step.  One workgroup per problem.  A column
// stops when it converges, when rz is not finite, or (max_iter > 0) after
// max_iter steps of the current solve.  Convergence is measured against the
// column's own energy E = (x_lin + u)^T K (x_lin + u) (its running estimate,
// from `esrc` when given, else from the column itself; at most the linear-field
// energy eref, at least 1e-6 eref): rz <= rtol2 E, or with use_init
// rz <= rtol2 min(rz_init, E).  Relative to E, the error of the energy-form
// average stays small against the homogenised value itself, also in the soft
// directions of a degraded matrix, where E is far below eref.  With loose > 0
// (inner FP32 passes of a refinement) the relative tolerance is raised to
// loose * eref / E where that is larger (at most 0.05): the accuracy an FP32
// operator can reach for the column.
template <int C, int R>
__global__ __launch_bounds__(512) void finish_beta_kernel(const Geo *geos, const Prob *probs, int NR, double *accbuf,
                                                         const double *ginv, double *ycoef, ColState *cols,
                                                         int *prob_active, int first, double rtol2, int use_init,
                                                         const ColState *mask, int max_iter, const ColState *esrc,
                                                         double loose) {
    constexpr int SMAX = C * 4;
    constexpr int RECMAX = ACC_RECMAX<C>;
    const int prob = blockIdx.x;
    const int nrow = geos[probs[prob].geo].nrow;
    const int REC = 2 + C * NR;
    const int S = C * nrow;
    const int lane = threadIdx.x;
    __shared__ double vals[R * RECMAX * ACC_STRIPES];
    __shared__ double sums[R * RECMAX];
    __shared__ double sG[SMAX * SMAX];
    __shared__ double sy[R * SMAX];
    __shared__ int sdone[R];
    double *base = accbuf + (long long)prob * R * RECMAX * ACC_STRIPES;
    for (int t = lane; t < R * RECMAX * ACC_STRIPES; t += blockDim.x) {
        vals[t] = base[t];
        base[t] = 0.0;
    }
    for (int k = lane; k < S * S; k += blockDim.x) sG[k] = ginv[(long long)prob * SMAX * SMAX + k];
    // coefficients of rows the problem does not have stay zero
    for (int k = lane; k < R * C * NR; k += blockDim.x) ycoef[(long long)prob * R * C * NR + k] = 0.0;
    __syncthreads();
    for (int e = lane; e < R * RECMAX; e += blockDim.x) {
        double v = 0.0;
        for (int st = 0; st < ACC_STRIPES; ++st) v += vals[e * ACC_STRIPES + st];
        sums[e] = v;
    }
    __syncthreads();
    // y = (C M^-1 C^T)^-1 c: one thread per (load case, row) entry
    if (lane < R * S) {
        const int w = lane / S, I = lane - (lane / S) * S;
        const double *rec = &sums[w * RECMAX];
        double t = 0.0;
        for (int J = 0; J < S; ++J) t += sG[I * S + J] * rec[2 + (J / nrow) * NR + (J % nrow)];
        sy[w * SMAX + I] = t;
        ycoef[((long long)prob * R + w) * C * NR + (I / nrow) * NR + (I % nrow)] = t;
    }
    __syncthreads();
    if (lane < R) {
        ColState &cs = cols[prob * R + lane];
        const double *rec = &sums[lane * RECMAX];
        double rz = rec[0];
        if (S > 0) {
            double cy = 0.0;
            for (int I = 0; I < S; ++I) cy += rec[2 + (I / nrow) * NR + (I % nrow)] * sy[lane * SMAX + I];
            rz -= cy;
            // r.Br - (CBr).y cancels: a projected part at the rounding level of
            // the sums cannot be resolved further (a homogeneous RVE under
            // uniform traction starts there: its right side lies in the range of
            // C^T), so the column counts as converged instead of iterating on noise
            if (rz <= 1e-13 * fabs(rec[0])) rz = 0.0;
        }
        if (rz < 0.0) rz = 0.0;
        const bool was_active = !cs.done;
        if (first) {
            cs.rz_init = rz;
            cs.beta = 0.0;
            cs.alpha = 0.0;   // no pending x update (see cg_dir_kernel)
            cs.done = (mask != nullptr && mask[prob * R + lane].done) ? COL_CONVERGED : COL_ACTIVE;
            cs.iters0 = cs.iters;
            if (!(cs.energy > 0.0)) cs.energy = cs.eref;   // start of the call: no CG step taken yet
        } else {
            cs.beta = (cs.done || cs.rz == 0.0) ? 0.0 : rz / cs.rz;
            if (was_active) cs.iters += 1;
        }
        if (first || was_active) {   // a stopped column keeps the residual it stopped with
            cs.rz_prev = cs.rz;
            cs.rz = rz;
        }
        double en = esrc != nullptr ? esrc[prob * R + lane].energy : cs.energy;
        if (!(en > 0.0)) en = cs.eref;
        en = fmin(fmax(en, 1e-6 * cs.eref), cs.eref);
        const double ref = use_init ? fmin(cs.rz_init, en) : en;
        const double rs = probs[prob].rtol2_scale;
        double tol2 = rs > 0.0 ? rtol2 * rs : rtol2;
        if (use_init && loose > 0.0) {
            const double t = fmin(loose * cs.eref / en, 0.05);
            tol2 = fmax(tol2, t * t);
        }
        if (!cs.done && !isfinite(rz)) cs.done = COL_NONFINITE;
        if (!cs.done && rz <= tol2 * ref) cs.done = COL_CONVERGED;
        if (!cs.done && !first && max_iter > 0 && cs.iters - cs.iters0 >= max_iter) cs.done = COL_CAPPED;
        if (cs.done) cs.beta = 0.0;
        sdone[lane] = cs.done;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int act = 0;
        for (int rr = 0; rr < R; ++rr) act += sdone[rr] ? 0 : 1;
        prob_active[prob] = act;
    }
}

// ------------------------------------------------------------------ launchers
#define CHOM_NR_DISPATCH(NRV, CALL)                    \
    switch (NRV) {                                     \
        case 0: { constexpr int NR = 0; CALL; } break; \
        case 1: { constexpr int NR = 1; CALL; } break; \
        default: { constexpr int NR = 4; CALL; } break; \
    }

template <typename T, int C, int R>
hipError_t launch_cg_init(const Launch &L, const T *b, T *x, T *r, const void *minv, double *accbuf, hipStream_t s) {
    dim3 grid(L.nwg, L.nprob);
    const T *M = (const T *)minv;
    if (x == nullptr) {
        CHOM_NR_DISPATCH(L.nr, (cg_init_kernel<T, C, R, NR, false><<<grid, 64 * R, 0, s>>>(L.geos, L.probs, b, x, r, M, accbuf)));
    } else {
        CHOM_NR_DISPATCH(L.nr, (cg_init_kernel<T, C, R, NR, true><<<grid, 64 * R, 0, s>>>(L.geos, L.probs, b, x, r, M, accbuf)));
    }
    return hipGetLastError();
}

template <typename T, int C, int R>
hipError_t launch_cg_dir(const Launch &L, T *x, T *r, T *p, const void *minv, const double *ycoef,
                         const ColState *cols, const int *prob_active, hipStream_t s, const void *mg_x0,
                         const void *mg_W) {
    dim3 grid(L.nwg, L.nprob);
    const T *M = (const T *)minv;
    MgDir<T> mg{(const T *)mg_x0, (const T *)mg_W, mg_x0 != nullptr ? 1 : 0};
    constexpr int KG = R % 2 == 0 ? 2 : (R % 3 == 0 ? 3 : 1);   // load cases per lane
    CHOM_NR_DISPATCH(L.nr, (cg_dir_kernel<T, C, R, NR, KG><<<grid, 64 * (R / KG), 0, s>>>(L.geos, L.probs, x, r, p, M, ycoef, cols, prob_active, mg)));
    return hipGetLastError();
}

template <typename T, int C, int R>
hipError_t launch_cg_update(const Launch &L, T *r, const T *q, const void *minv, const ColState *cols,
                            double *accbuf, const int *prob_active, hipStream_t s) {
    dim3 grid(L.nwg, L.nprob);
    const T *M = (const T *)minv;
    // each wave takes KG load cases of one operator group: KG = 3 or 2 when it
    // divides the group size L.rg, else 1
    if (L.rg % 3 == 0 && R % 3 == 0) {
        constexpr int KG = R % 3 == 0 ? 3 : 1;
        CHOM_NR_DISPATCH(L.nr, (cg_update_kernel<T, C, R, NR, KG><<<grid, 64 * (R / KG), 0, s>>>(
                                   L.geos, L.probs, L.rg, r, q, M, cols, accbuf, prob_active)));
    } else if (L.rg % 2 == 0 && R % 2 == 0) {
        constexpr int KG = R % 2 == 0 ? 2 : 1;
        CHOM_NR_DISPATCH(L.nr, (cg_update_kernel<T, C, R, NR, KG><<<grid, 64 * (R / KG), 0, s>>>(
                                   L.geos, L.probs, L.rg, r, q, M, cols, accbuf, prob_active)));
    } else {
        CHOM_NR_DISPATCH(L.nr, (cg_update_kernel<T, C, R, NR, 1><<<grid, 64 * R, 0, s>>>(
                                   L.geos, L.probs, L.rg, r, q, M, cols, accbuf, prob_active)));
    }
    return hipGetLastError();
}

template <typename T, int C, int R>
hipError_t launch_cg_flush_x(const Launch &L, T *x, const T *p, const ColState *cols, hipStream_t s) {
    cg_flush_x_kernel<T, C, R><<<dim3(L.nwg, L.nprob), 64 * R, 0, s>>>(L.geos, L.probs, x, p, cols);
    return hipGetLastError();
}

template <int C, int R>
hipError_t launch_proj_resid(const Launch &L, double *r64, float *r32, const double *minv64,
                             const double *ycoef, double *partial, hipStream_t s) {
    dim3 grid(L.nwg, L.nprob);
    CHOM_NR_DISPATCH(L.nr, (proj_resid_kernel<C, R, NR><<<grid, 64 * R, 0, s>>>(L.geos, L.probs, r64, r32, minv64, ycoef, partial)));
    return hipGetLastError();
}

template <int C, int R>
hipError_t launch_finish_alpha(const Launch &L, double *acc_pq, ColState *cols, hipStream_t s) {
    finish_alpha_kernel<R><<<L.nprob, 256, 0, s>>>(acc_pq, cols);
    return hipGetLastError();
}

template <int C, int R>
hipError_t launch_finish_beta(const Launch &L, double *accbuf, const double *ginv, double *ycoef, ColState *cols,
                              int *prob_active, int first, double rtol2, int use_init, const ColState *mask,
                              hipStream_t s, int max_iter, const ColState *esrc, double loose) {
    finish_beta_kernel<C, R><<<L.nprob, 512, 0, s>>>(L.geos, L.probs, L.nr, accbuf, ginv, ycoef, cols, prob_active,
                                                    first, rtol2, use_init, mask, max_iter, esrc, loose);
    return hipGetLastError();
}

__global__ void zero_kernel(long long n, double *p) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

hipError_t launch_zero(double *p, long long n, hipStream_t s) {
    long long g = (n + 255) / 256;
    zero_kernel<<<(int)(g < 1024 ? (g < 1 ? 1 : g) : 1024), 256, 0, s>>>(n, p);
    return hipGetLastError();
}

// ------------------------------------------------------------------ refinement helpers
template <int C, int R>
__global__ void residual64_kernel(const Geo *geos, const Prob *probs, int rg, const double *b, const double *q64t,
                                  double *r64, float *r32) {
    const int prob = blockIdx.y;
    const Prob &P = probs[prob];
    const Geo &G = geos[P.geo];
    const double *qt = q64t ? q64t + P.qoff : nullptr;
    for (long long pt = blockIdx.x * (long long)blockDim.x + threadIdx.x; pt < G.npts;
         pt += (long long)gridDim.x * blockDim.x) {
        int X, Y, Z;
        lattice_xyz(G, pt, X, Y, Z);
        const bool gather = qt != nullptr && !dirichlet_boundary(G, X, Y, Z);
        for (int w = 0; w < R; ++w) {   // one load case at a time: few live registers
            double qv[C];
#pragma unroll
            for (int c = 0; c < C; ++c) qv[c] = 0.0;
            if (gather) gather_tiles_col<double, C, R>(G, qt, rg, X, Y, Z, w, qv);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const long long o = P.voff + ((long long)w * G.npts + pt) * C + c;
                const double val = (b ? b[o] : 0.0) - qv[c];
                r64[o] = val;
                if (r32) r32[o] = (float)val;
            }
        }
    }
}

template <int C, int R>
hipError_t launch_residual64(const Launch &L, const double *b, const double *q64t, double *r64, float *r32,
                             hipStream_t s) {
    dim3 grid(L.nwg, L.nprob);
    residual64_kernel<C, R><<<grid, 256, 0, s>>>(L.geos, L.probs, L.rg, b, q64t, r64, r32);
    return hipGetLastError();
}

__global__ void axpy_x64_kernel(long long total, double *x64, const float *d32) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x)
        x64[i] += (double)d32[i];
}

hipError_t launch_axpy_x64(long long total, double *x64, const float *d32, hipStream_t s) {
    long long g = (total + 255) / 256;
    g = g < 1 ? 1 : (g > 16384 ? 16384 : g);
    axpy_x64_kernel<<<(int)g, 256, 0, s>>>(total, x64, d32);
    return hipGetLastError();
}

__global__ void axpy64_kernel(long long total, double *x64, const double *d64) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x)
        x64[i] += d64[i];
}

hipError_t launch_axpy64(long long total, double *x64, const double *d64, hipStream_t s) {
    long long g = (total + 255) / 256;
    g = g < 1 ? 1 : (g > 16384 ? 16384 : g);
    axpy64_kernel<<<(int)g, 256, 0, s>>>(total, x64, d64);
    return hipGetLastError();
}

// Projection of the FP64 solution onto ker(C): x -= M^-1 C^T (C M^-1 C^T)^-1 C x.
// Partial layout (k-major): [prob][R][C * 4][nwg].
template <int C, int R>
__global__ void cx_partial_kernel(const Geo *geos, const Prob *probs, const double *x, double *partial) {
    constexpr int S4 = C * 4;
    const int prob = blockIdx.y;
    const Prob &P = probs[prob];
    const Geo &G = geos[P.geo];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nr = G.nrow, rf = row_first(G.nrow);
    double acc[S4];
    for (int k = 0; k < S4; ++k) acc[k] = 0.0;
    const long long nblk = (G.npts + 63) / 64;
    for (long long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const long long pt = blk * 64 + lane;
        if (pt >= G.npts) continue;
        const long long o = P.voff + (w * G.npts + pt) * C;
        for (int a = 0; a < nr; ++a) {
            const double rw = G.rows[4 * pt + rf + a];
            for (int c = 0; c < C; ++c) acc[c * 4 + a] += rw * x[o + c];
        }
    }
    wave_partials<S4>(acc, partial, prob, R, w);
}

template <int C, int R>
__global__ void cx_finish_kernel(const Geo *geos, const Prob *probs, const double *partial, int nparts,
                                 const double *ginv, double *ycoef) {
    constexpr int S4 = C * 4;
    const int prob = blockIdx.x;
    const int nrow = geos[probs[prob].geo].nrow;
    __shared__ double sums[R * S4];
    reduce_kmajor(partial + (long long)prob * R * S4 * nparts, R * S4, nparts, sums);
    __syncthreads();
    const int lane = threadIdx.x;
    if (lane < R) {
        const int S = C * nrow;
        const double *Gi = ginv + (long long)prob * S4 * S4;
        double *yv = ycoef + ((long long)prob * R + lane) * S4;
        for (int k = 0; k < S4; ++k) yv[k] = 0.0;
        for (int I = 0; I < S; ++I) {
            double t = 0.0;
            for (int J = 0; J < S; ++J) t += Gi[I * S + J] * sums[lane * S4 + (J / nrow) * 4 + (J % nrow)];
            yv[(I / nrow) * 4 + (I % nrow)] = t;
        }
    }
}

template <int C, int R>
__global__ void cx_correct_kernel(const Geo *geos, const Prob *probs, double *x, const double *minv64,
                                  const double *ycoef) {
    constexpr int MS = (C == 3) ? 6 : 1;
    constexpr int S4 = C * 4;
    const int prob = blockIdx.y;
    const Prob &P = probs[prob];
    const Geo &G = geos[P.geo];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nr = G.nrow, rf = row_first(G.nrow);
    if (nr == 0) return;
    const double *yv = ycoef + ((long long)prob * R + w) * S4;
    const long long nblk = (G.npts + 63) / 64;
    for (long long blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const long long pt = blk * 64 + lane;
        if (pt >= G.npts) continue;
        double Mi[MS];
        for (int k = 0; k < MS; ++k) Mi[k] = minv64[(P.doff + pt) * MS + k];
        double ct[C], corr[C];
        for (int c = 0; c < C; ++c) {
            ct[c] = 0.0;
            for (int a = 0; a < nr; ++a) ct[c] += G.rows[4 * pt + rf + a] * yv[c * 4 + a];
        }
        minv_apply<double, C>(Mi, ct, corr);
        const long long o = P.voff + (w * G.npts + pt) * C;
        for (int c = 0; c < C; ++c) x[o + c] -= corr[c];
    }
}

template <int C, int R>
hipError_t launch_project(const Launch &L, double *x64, const double *minv64, const double *ginv64,
                          double *partial, hipStream_t s) {
    if (L.nr == 0) return hipSuccess;
    dim3 grid(L.nwg, L.nprob);
    double *ycoef = partial + (long long)L.nprob * L.nwg * R * C * 4;
    cx_partial_kernel<C, R><<<grid, 64 * R, 0, s>>>(L.geos, L.probs, x64, partial);
    cx_finish_kernel<C, R><<<L.nprob, 256, 0, s>>>(L.geos, L.probs, partial, L.nwg, ginv64, ycoef);
    cx_correct_kernel<C, R><<<grid, 64 * R, 0, s>>>(L.geos, L.probs, x64, minv64, ycoef);
    return hipGetLastError();
}

// ------------------------------------------------------------------ instantiations
#define CHOM_INST(T, C, R)                                                                                        \
    template hipError_t launch_cg_init<T, C, R>(const Launch &, const T *, T *, T *, const void *, double *,      \
                                                hipStream_t);                                                    \
    template hipError_t launch_cg_dir<T, C, R>(const Launch &, T *, T *, T *, const void *, const double *,      \
                                               const ColState *, const int *, hipStream_t, const void *,         \
                                               const void *);                                                    \
    template hipError_t launch_cg_update<T, C, R>(const Launch &, T *, const T *, const void *, const ColState *, \
                                                  double *, const int *, hipStream_t);                           \
    template hipError_t launch_cg_flush_x<T, C, R>(const Launch &, T *, const T *, const ColState *, hipStream_t);
CHOM_INST(double, 3, 6)
CHOM_INST(float, 3, 6)
CHOM_INST(double, 1, 3)
CHOM_INST(float, 1, 3)

#define CHOM_INST2(C, R)                                                                                         \
    template hipError_t launch_finish_alpha<C, R>(const Launch &, double *, ColState *, hipStream_t);            \
    template hipError_t launch_finish_beta<C, R>(const Launch &, double *, const double *, double *, ColState *, \
                                                 int *, int, double, int, const ColState *, hipStream_t, int,    \
                                                 const ColState *, double);                                      \
    template hipError_t launch_proj_resid<C, R>(const Launch &, double *, float *, const double *,               \
                                                const double *, double *, hipStream_t);                          \
    template hipError_t launch_residual64<C, R>(const Launch &, const double *, const double *, double *, float *, \
                                                hipStream_t);                                                    \
    template hipError_t launch_project<C, R>(const Launch &, double *, const double *, const double *, double *,  \
                                             hipStream_t);
CHOM_INST2(3, 6)
CHOM_INST2(1, 3)

}  // namespace chom
