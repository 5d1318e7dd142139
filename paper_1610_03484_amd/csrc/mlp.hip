// Learned surrogate of the homogenisation map: an ensemble of small MLPs
// (10 features -> 256 -> 256 -> 256 -> 36, GELU hidden layers; the 36 outputs
// encode C_bar, K_bar, D_bar per block as log-norm and direction), trained and
// evaluated by the kernels in this file.
//
// Features of a record (T, c, t, 8 factors): log(1 - omega), (1 - omega) and the
// factors, with (1 - omega) = exp(-gamma(c) alpha(T) t) the constant-exposure
// degradation law of Sec. 4 (Eq. Eq_Model_final1), alpha = beta ln(1 - T/T_g)
// in kelvin (Eq. Eq_alphaT), gamma = c / c_sat, t in days.
//
// Precision: weights and activations are bfloat16 in the products, which run on
// the matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulate); biases, pre-
// activations, the loss, gradients and the Adam state are FP32; feature
// standardisation and the final de-standardisation are FP64.
//
// Training: each member's minibatch step is spread over eight workgroups that
// split every hidden layer by columns (details at the training kernels); all
// members run in the same launches.  Activations of the minibatch live in a
// per-member global scratch; each is stored row-major for the next layer's
// product and transposed for the weight-gradient product, so that both operands
// of every product are contiguous along the contraction.
//
// Inference: one workgroup per 64 points evaluates every member with the
// activations in LDS and keeps the ensemble mean and variance in registers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp.h"

namespace chom {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// The same rounding (to nearest, ties to even) by the hardware conversion; finite values only.
__device__ __forceinline__ uint16_t to_bf16_hw(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// Standard normal distribution function Phi(z) = erfc(-z / sqrt 2) / 2, with erfc
// from the Chebyshev fit published in Numerical Recipes (Press, Teukolsky,
// Vetterling, Flannery; function erfcc: fractional error below 1.2e-7 for every
// argument), one hardware reciprocal and one hardware exponential: far cheaper on
// the vector units than a general-purpose erf, and exact to well below the
// bfloat16 rounding the activations then take.
__device__ __forceinline__ float norm_cdf(float z) {
    const float x = fabsf(z) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(1.0f + 0.5f * x);
    const float q = 1.00002368f +
                    t * (0.37409196f +
                         t * (0.09678418f +
                              t * (-0.18628806f +
                                   t * (0.27886807f +
                                        t * (-1.13520398f + t * (1.48851587f + t * (-0.82215223f + t * 0.17087277f)))))));
    const float ec = t * __expf(-x * x - 1.26551223f + t * q);   // erfc(x)
    return z >= 0.0f ? 1.0f - 0.5f * ec : 0.5f * ec;
}
__device__ __forceinline__ float gelu(float z) { return z * norm_cdf(z); }
__device__ __forceinline__ float gelu_grad(float z) {
    return norm_cdf(z) + z * __expf(-0.5f * z * z) * 0.39894228040143268f;
}

// Features of one record; false when the record is outside the law's domain.
__device__ __forceinline__ bool record_features(const double *rec, double c_sat, double f[NF]) {
    const double TK = rec[0] + KELVIN, TgK = TG_CELSIUS + KELVIN;
    const double arg = 1.0 - TK / TgK;
    if (!(arg > 0.0) || !(rec[1] >= 0.0) || !(rec[2] >= 0.0)) return false;
    const double alpha = BETA * log(arg);
    const double gamma = rec[1] / c_sat;
    const double t_days = rec[2] * DAYS_PER_YEAR;
    const double lk = -gamma * alpha * t_days;
    f[0] = lk;
    f[1] = exp(lk);
    for (int k = 0; k < 8; ++k) {
        f[2 + k] = rec[3 + k];
        if (!(rec[3 + k] > 0.0)) return false;
    }
    return true;
}

// Output encoding.  Network column k: 0 log||C||, 1..21 C / ||C||, 22 log||K||,
// 23..28 K / ||K||, 29 log||D||, 30..35 D / ||D||; ||.|| is the Frobenius norm of
// the full symmetric matrix (off-diagonal entries of the upper triangle count twice).
__host__ __device__ constexpr int col_block(int col) { return col < 22 ? 0 : (col < 29 ? 1 : 2); }
__host__ __device__ constexpr bool col_is_log(int col) { return col == 0 || col == 22 || col == 29; }
__host__ __device__ constexpr int col_phys(int col) { return col - 1 - col_block(col); }
__host__ __device__ inline float phys_weight(int p) {
    if (p < 21) {   // upper triangle row-major: diagonal entries at 0, 6, 11, 15, 18, 20
        return (p == 0 || p == 6 || p == 11 || p == 15 || p == 18 || p == 20) ? 1.0f : 2.0f;
    }
    const int k = p < 27 ? p - 21 : p - 27;
    return k < 3 ? 1.0f : 2.0f;
}

// Physical output p (0..32) of record i.
__device__ __forceinline__ double phys_value(const double *C, const double *K, const double *D, long long i, int p) {
    return p < 21 ? C[i * 21 + p] : (p < 27 ? K[i * 6 + p - 21] : D[i * 6 + p - 27]);
}

// Encoded column col of record i (FP64).
__device__ double encoded_value(const double *C, const double *K, const double *D, long long i, int col) {
    const int b = col_block(col);
    const int p0 = b == 0 ? 0 : (b == 1 ? 21 : 27), p1 = b == 0 ? 21 : (b == 1 ? 27 : 33);
    double s = 0.0;
    for (int p = p0; p < p1; ++p) {
        const double v = phys_value(C, K, D, i, p);
        s += (double)phys_weight(p) * v * v;
    }
    const double nrm = sqrt(s);
    return col_is_log(col) ? log(nrm) : phys_value(C, K, D, i, col_phys(col)) / nrm;
}

// One wave: acc[i][j] += A[16i.., :K] * B[16j.., :K]^T for 16x16 tiles; A and B are
// bfloat16, row-major with the contraction index contiguous (row strides lda, ldb).
// Lane l supplies row (l & 15) and the 8 contraction entries starting at 8 (l >> 4)
// of each operand tile; the result element (4 (l >> 4) + q, l & 15) of tile (i, j)
// lands in acc[i][j][q].
//
// FULL unrolls the contraction completely, so that every operand load is issued
// before the first product (for operands that come from memory written by the
// previous kernel, whose latency would otherwise be paid once per step of 32).
template <int TM, int TN, int K, bool FULL = false>
__device__ __forceinline__ void wave_mma(const uint16_t *__restrict__ A, int lda, const uint16_t *__restrict__ B,
                                         int ldb, f32x4 (&acc)[TM][TN]) {
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, kq = (lane >> 4) << 3;
    const uint16_t *Ap = A + r * lda + kq;
    const uint16_t *Bp = B + r * ldb + kq;
#pragma unroll FULL ? K / 32 : 2
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
            a[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(Ap + 16 * i * lda + k0));
#pragma unroll
        for (int j = 0; j < TN; ++j)
            b[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(Bp + 16 * j * ldb + k0));
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
}

template <int TM, int TN>
__device__ __forceinline__ void zero_acc(f32x4 (&acc)[TM][TN]) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// ------------------------------------------------------------------ per-member views
struct MemberW {   // weights of one member
    float *w, *m, *v;                           // FP32 master and Adam moments, flat layout
    uint16_t *w1b, *w2b, *w3b, *w4b, *w2t, *w3t, *w4t;
};

__device__ __forceinline__ MemberW member_weights(const Weights &W, int mem) {
    MemberW o;
    o.w = W.master + (size_t)mem * NPARAM;
    o.m = W.adam_m + (size_t)mem * NPARAM;
    o.v = W.adam_v + (size_t)mem * NPARAM;
    o.w1b = W.w1b + (size_t)mem * H * FP;
    o.w2b = W.w2b + (size_t)mem * H * H;
    o.w3b = W.w3b + (size_t)mem * H * H;
    o.w4b = W.w4b + (size_t)mem * OP * H;
    o.w2t = W.w2t + (size_t)mem * H * H;
    o.w3t = W.w3t + (size_t)mem * H * H;
    o.w4t = W.w4t + (size_t)mem * H * OP;
    return o;
}

// ------------------------------------------------------------------ bf16 copies of the master weights
// For every member: w1b [H][FP] (columns >= NF zero), w2b/w3b [H][H], w4b [OP][H]
// (rows >= NO zero) and the transposes w2t/w3t [H][H], w4t [H][OP].
__global__ void sync_bf16_kernel(Weights W, int members) {
    const long long per = (long long)H * FP + 2LL * H * H + (long long)OP * H;
    const long long total = per * members;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int mem = (int)(e / per);
        long long r = e - mem * per;
        const float *w = W.master + (size_t)mem * NPARAM;
        if (r < H * FP) {
            const int o = (int)(r / FP), i = (int)(r % FP);
            const uint16_t v = i < NF ? to_bf16(w[OFF_W1 + o * NF + i]) : (uint16_t)0;
            W.w1b[(size_t)mem * H * FP + r] = v;
            continue;
        }
        r -= H * FP;
        if (r < 2LL * H * H) {
            const int l = (int)(r / (H * H));
            const int rr = (int)(r % (H * H));
            const int o = rr / H, i = rr % H;
            const uint16_t v = to_bf16(w[(l == 0 ? OFF_W2 : OFF_W3) + rr]);
            (l == 0 ? W.w2b : W.w3b)[(size_t)mem * H * H + rr] = v;
            (l == 0 ? W.w2t : W.w3t)[(size_t)mem * H * H + i * H + o] = v;
            continue;
        }
        r -= 2LL * H * H;
        {
            const int o = (int)(r / H), i = (int)(r % H);
            const uint16_t v = o < NO ? to_bf16(w[OFF_W4 + o * H + i]) : (uint16_t)0;
            W.w4b[(size_t)mem * OP * H + r] = v;
            W.w4t[(size_t)mem * H * OP + i * OP + o] = v;
        }
    }
}

// ------------------------------------------------------------------ standardisation statistics
// One workgroup per column: columns 0..NF-1 are features, NF..NF+NO-1 the
// encoded outputs.  Mean and population deviation in FP64 (1 when zero).
__global__ __launch_bounds__(256) void stats_kernel(const double *params, const double *C, const double *K,
                                                   const double *D, long long n, double c_sat, double *norm,
                                                   int *bad) {
    const int col = blockIdx.x;
    __shared__ double red[256];
    __shared__ double s_mean;
    auto value = [&](long long i, bool &ok) -> double {
        ok = true;
        if (col < NF) {
            double f[NF];
            ok = record_features(params + i * 11, c_sat, f);
            return f[col];
        }
        return encoded_value(C, K, D, i, col - NF);
    };
    double s = 0.0;
    for (long long i = threadIdx.x; i < n; i += 256) {
        bool ok;
        const double v = value(i, ok);
        if (!ok || !isfinite(v)) atomicOr(bad, 1);
        else s += v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) s_mean = red[0] / (double)n;
    __syncthreads();
    const double mu = s_mean;
    double q = 0.0;
    for (long long i = threadIdx.x; i < n; i += 256) {
        bool ok;
        const double v = value(i, ok);
        if (ok && isfinite(v)) q += (v - mu) * (v - mu);
    }
    __syncthreads();
    red[threadIdx.x] = q;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double sd = sqrt(red[0] / (double)n);
        const int mcol = col < NF ? col : col - NF;
        double *mean_out = col < NF ? norm + NORM_XMU : norm + NORM_YMU;
        double *sd_out = col < NF ? norm + NORM_XSD : norm + NORM_YSD;
        mean_out[mcol] = mu;
        sd_out[mcol] = sd > 0.0 ? sd : 1.0;
    }
}

// Standardised training rows: xn [n][FP] bfloat16 (zero padded), tn [n][NO] FP32
// (encoded outputs).
__global__ void prepare_kernel(const double *params, const double *C, const double *K, const double *D, long long n,
                               double c_sat, const double *norm, uint16_t *xn, float *tn, int *bad) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double f[NF];
        if (!record_features(params + i * 11, c_sat, f)) atomicOr(bad, 1);
        for (int k = 0; k < FP; ++k) {
            uint16_t v = 0;
            if (k < NF) v = to_bf16((float)((f[k] - norm[NORM_XMU + k]) / norm[NORM_XSD + k]));
            xn[i * FP + k] = v;
        }
        for (int o = 0; o < NO; ++o) {
            const double y = encoded_value(C, K, D, i, o);
            if (!isfinite(y)) atomicOr(bad, 1);
            tn[i * NO + o] = (float)((y - norm[NORM_YMU + o]) / norm[NORM_YSD + o]);
        }
    }
}

// ------------------------------------------------------------------ training
// A minibatch step of one member is spread over NSL workgroups, workgroup j
// owning hidden columns [SL j, SL j + SL) of every layer: it forms those columns
// of the layer's output for all rows, and the weight rows of those outputs are
// its alone -- their gradient (the product of its own output-gradient columns
// with the full input activations), their Adam state and their update.  Only
// whole activations and output gradients cross workgroups, through the
// member's scratch, so a step is five kernels in order:
//   F2, F3      hidden layers 2 and 3 (layer 1 runs at the end of the previous step)
//   B3          output layer and loss (every workgroup, redundantly), output-layer
//               weight columns, layer-3 gradient columns, layer-3 weight rows
//   B2          layer-2 gradient columns and weight rows (and the output bias)
//   B1F1        layer-1 gradient columns and weight rows, then layer 1 of the
//               next step with the updated rows
// A step reads the bfloat16 weight copies of set (step & 1) and writes the
// updated copies into the other set, so no kernel reads a copy that another
// workgroup of the same step is rewriting.  Each kernel reads its step index
// from a counter of its own that the previous kernel of the sequence set, so a
// graph of several steps can be replayed unchanged.
constexpr int K_F2 = 0, K_F3 = 1, K_B3 = 2, K_B2 = 3, K_B1 = 4;
static_assert(TRAIN_THREADS % 64 == 0 && TRAIN_THREADS / 64 == 8 && TRAIN_THREADS >= NB, "eight waves; a thread per row");
// LDS row strides (bfloat16 elements), padded so that the 16 rows an MFMA
// operand load touches fall on different banks.
constexpr int GTS = NB + 8;    // transposed gradient tiles [.][NB]
constexpr int G4S = OP + 8;    // output gradient [NB][OP]
constexpr int X1S = FP + 8;    // features [NB][FP]

struct BfView {
    uint16_t *w1b, *w2b, *w3b, *w4b, *w2t, *w3t, *w4t;
};

__device__ __forceinline__ BfView bf_view(const Weights &W, int mem, int set) {
    BfView v;
    if (set == 0) {
        v.w1b = W.w1b + (size_t)mem * H * FP;
        v.w2b = W.w2b + (size_t)mem * H * H;
        v.w3b = W.w3b + (size_t)mem * H * H;
        v.w4b = W.w4b + (size_t)mem * OP * H;
        v.w2t = W.w2t + (size_t)mem * H * H;
        v.w3t = W.w3t + (size_t)mem * H * H;
        v.w4t = W.w4t + (size_t)mem * H * OP;
    } else {
        uint16_t *b = W.alt + (size_t)mem * BF_PER_MEMBER;
        v.w1b = b;
        v.w2b = v.w1b + H * FP;
        v.w3b = v.w2b + H * H;
        v.w4b = v.w3b + H * H;
        v.w2t = v.w4b + OP * H;
        v.w3t = v.w2t + H * H;
        v.w4t = v.w3t + H * H;
    }
    return v;
}

template <typename T> __device__ __forceinline__ T *sp(unsigned char *base, long long off) {
    return reinterpret_cast<T *>(base + off);
}
#define S_A(l) sp<uint16_t>(sb, MS_A + (l) * (long long)NB * H * 2)
#define S_AT(l) sp<uint16_t>(sb, MS_AT + (l) * (long long)NB * H * 2)
#define S_D(l) sp<float>(sb, MS_D + (l) * (long long)NB * H * 4)
#define S_G(l) sp<uint16_t>(sb, MS_G + (l) * (long long)NB * H * 2)   // l = 0: layer 3, 1: layer 2
#define S_B4G sp<float>(sb, MS_B4G)
#define S_LOSS sp<double>(sb, MS_LOSS)

struct AdamC {
    float lr, b1, b2, eps, bc1, bc2;
};

__device__ __forceinline__ void adam_update(float &w, float &m, float &v, float g, const AdamC &c) {
    m = c.b1 * m + (1.0f - c.b1) * g;
    v = c.b2 * v + (1.0f - c.b2) * g * g;
    w = w - c.lr * (m / c.bc1) / (sqrtf(v / c.bc2) + c.eps);
}

__device__ __forceinline__ long long perm_index(long long i, long long n, long long a, long long b) {
    // affine bijection of [0, n): gcd(a, n) = 1
    // a, i < n < 2^31: the product fits in 64 bits
    return (long long)(((unsigned long long)a * (unsigned long long)i + (unsigned long long)b) % (unsigned long long)n);
}

__device__ __forceinline__ uint64_t splitmix(uint64_t state) {
    uint64_t z = state + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ long long gcd_ll(long long a, long long b) {
    while (b) {
        const long long t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Where step g of the sequence stands: its epoch, its position in the epoch
// and its rows.
struct StepPos {
    long long g, ep, st, i0, steps, total;
    int nbe;
};

__device__ __forceinline__ StepPos step_pos(const TrainArgs &A, long long g) {
    StepPos c;
    c.g = g;
    c.steps = (A.n + A.nb - 1) / A.nb;
    c.total = c.steps * (long long)A.epochs;
    c.ep = g / c.steps;
    c.st = g - c.ep * c.steps;
    c.i0 = c.st * A.nb;
    c.nbe = (int)min((long long)A.nb, A.n - c.i0);
    return c;
}

// Source rows of step c's minibatch into src[NB] (LDS; -1 past the rows of the
// step).  The epoch's shuffle is an affine bijection drawn from the member's
// stream when the epoch starts (and kept in the member's scratch by workgroup 0
// for the rest of the epoch).  Every thread of the workgroup must call this.
__device__ void step_rows(const TrainArgs &A, int mem, const StepPos &c, unsigned char *sb, int *src) {
    __shared__ long long s_pa, s_pb;
    long long *perm = reinterpret_cast<long long *>(sb + MS_PERM);
    __syncthreads();   // src and s_pa, s_pb of an earlier call are no longer read
    if (threadIdx.x == 0) {
        long long a = 1, b = 0;
        if (A.grad == nullptr && A.n > 1) {
            if (c.st == 0) {
                const uint64_t key = (A.seed << 32) + ((uint64_t)mem << 20) + (uint64_t)(A.epoch0 + c.ep);
                a = 1 + (long long)(splitmix(key) % (uint64_t)(A.n - 1));
                while (gcd_ll(a, A.n) != 1) a = a % (A.n - 1) + 1;      // ends: a = 1 is coprime
                b = (long long)(splitmix(key ^ 0x5DEECE66Dull) % (uint64_t)A.n);
                if (blockIdx.x == 0) {
                    perm[0] = a;
                    perm[1] = b;
                }
            } else {
                a = perm[0];
                b = perm[1];
            }
        }
        s_pa = a;
        s_pb = b;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < NB; r += TRAIN_THREADS)
        src[r] = r < c.nbe ? (int)perm_index(c.i0 + r, A.n, s_pa, s_pb) : -1;
    __syncthreads();
}

__device__ AdamC adam_constants(const TrainArgs &A, const StepPos &c) {
    AdamC a;
    const long long t = A.step0 + c.g + 1;
    const double frac = c.total > 1 ? (double)c.g / (double)(c.total - 1) : 1.0;
    const double lr = A.lr1 + 0.5 * (A.lr0 - A.lr1) * (1.0 + cos(3.14159265358979323846 * frac));
    a.lr = (float)lr;
    a.b1 = A.beta1;
    a.b2 = A.beta2;
    a.eps = A.eps;
    a.bc1 = (float)(1.0 - pow((double)A.beta1, (double)t));
    a.bc2 = (float)(1.0 - pow((double)A.beta2, (double)t));
    return a;
}

// Gradients of N parameters of a lane: accumulate them (gradient mode) or take
// an Adam step (the new master values are left in w).  Every load is issued
// before the first store, so the lane waits for memory once, not once per
// parameter.
template <int N>
__device__ __forceinline__ void apply_grads(const TrainArgs &A, const MemberW &M, const int (&off)[N],
                                            const float (&g)[N], const bool (&on)[N], const AdamC &c,
                                            float (&w)[N]) {
    if (A.grad != nullptr) {
#pragma unroll
        for (int k = 0; k < N; ++k) w[k] = on[k] ? A.grad[off[k]] : 0.f;
#pragma unroll
        for (int k = 0; k < N; ++k)
            if (on[k]) A.grad[off[k]] = w[k] + g[k];
        return;
    }
    float m[N], v[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        w[k] = on[k] ? M.w[off[k]] : 0.f;
        m[k] = on[k] ? M.m[off[k]] : 0.f;
        v[k] = on[k] ? M.v[off[k]] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
        if (!on[k]) continue;
        adam_update(w[k], m[k], v[k], g[k], c);
        M.w[off[k]] = w[k];
        M.m[off[k]] = m[k];
        M.v[off[k]] = v[k];
    }
}

__device__ __forceinline__ void apply_grad1(const TrainArgs &A, const MemberW &M, int off, float g, const AdamC &c) {
    const int o[1] = {off};
    const float gg[1] = {g};
    const bool on[1] = {true};
    float w[1];
    apply_grads<1>(A, M, o, gg, on, c, w);
}

// Sum over the NB rows of a transposed gradient row (bias gradient).
__device__ __forceinline__ float row_sum(const uint16_t *gt_row) {
    float s = 0.f;
#pragma unroll 4
    for (int r = 0; r < NB; r += 8) {
        const uint4 v = *reinterpret_cast<const uint4 *>(gt_row + r);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) s += from_bf16((uint16_t)(w[k] & 0xFFFF)) + from_bf16((uint16_t)(w[k] >> 16));
    }
    return s;
}

// The step counter of kernel k; the first workgroup hands the step on to the
// next kernel of the sequence (B1F1 hands on the next step).
__device__ __forceinline__ long long take_step(const TrainArgs &A, int k) {
    int *ctr = reinterpret_cast<int *>(A.scratch);
    const long long g = ctr[k];
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) ctr[(k + 1) % 5] = (int)g + (k == K_B1 ? 1 : 0);
    return g;
}

__device__ __forceinline__ unsigned char *member_scratch(const TrainArgs &A) {
    return A.scratch + TS_CTRL + (size_t)blockIdx.y * MEMBER_SCRATCH;
}

// Columns [SL j, SL j + SL) of a hidden layer for all NB rows: z = A W^T + b,
// written as a = gelu(z) (bfloat16, row-major and transposed) and gelu'(z).  A is
// [NB][K] with row stride lda; Wrows points at the first of the layer's weight
// rows SL j .. SL j + SL - 1 (row stride K).
template <int K>
__device__ __forceinline__ void fwd_slice(const uint16_t *A, int lda, const uint16_t *Wrows, const float *bias,
                                          int j, uint16_t *aout, uint16_t *atout, float *dout) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = 32 * wave;
    f32x4 acc[2][2];
    zero_acc(acc);
    wave_mma<2, 2, K, true>(A + m0 * lda, lda, Wrows, K, acc);
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
        const int col = SL * j + 16 * jj + (lane & 15);
        const float b = bias[col];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int row0 = m0 + 16 * i + 4 * (lane >> 4);
            uint16_t h[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float z = acc[i][jj][q] + b;
                h[q] = to_bf16(gelu(z));
                aout[(row0 + q) * H + col] = h[q];
                dout[(row0 + q) * H + col] = gelu_grad(z);
            }
            uint2 pk;
            pk.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
            pk.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
            *reinterpret_cast<uint2 *>(atout + col * NB + row0) = pk;
        }
    }
}

// Columns [SL j, SL j + SL) of a hidden layer's output gradient: g = bf16((G Wt^T) * gelu'(z)),
// G [NB][K] (stride ldg), Wt the transposed weights of the layer above (rows = this
// layer's columns, stride K).  Written transposed into gt [SL][GTS] (LDS) and, when
// grow is set, row-major into grow [NB][H].  The product is formed first; the
// barrier before the writes lets gt share memory with an operand.
template <int K>
__device__ __forceinline__ void bwd_slice(const uint16_t *G, int ldg, const uint16_t *Wt, const float *dprev, int j,
                                          uint16_t *grow, uint16_t *gt) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = 32 * wave;
    float dp[2][2][4];   // gelu'(z) of this lane's outputs, loaded with the operands
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                dp[jj][i][q] = dprev[(m0 + 16 * i + 4 * (lane >> 4) + q) * H + SL * j + 16 * jj + (lane & 15)];
    f32x4 acc[2][2];
    zero_acc(acc);
    wave_mma<2, 2, K, true>(G + m0 * ldg, ldg, Wt + SL * j * K, K, acc);
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
        const int cl = 16 * jj + (lane & 15);
        const int col = SL * j + cl;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int row0 = m0 + 16 * i + 4 * (lane >> 4);
            uint16_t h[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                h[q] = to_bf16(acc[i][jj][q] * dp[jj][i][q]);
                if (grow) grow[(row0 + q) * H + col] = h[q];
            }
            uint2 pk;
            pk.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
            pk.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
            *reinterpret_cast<uint2 *>(gt + cl * GTS + row0) = pk;
        }
    }
}

// The parameters of a lane in the weight-row update of a 256-wide hidden layer
// (wgrad_rows): lane l of wave w holds o = SL j + 16 i + 4 (l >> 4) + q,
// in = 32 w + 16 jj + (l & 15), entry (2 i + jj) 4 + q.  Their master values and
// Adam moments (or accumulated gradients) are loaded once, at the start of the
// kernel, so the update does not wait for memory.
struct RowState {
    float w[16], m[16], v[16];
};

__device__ __forceinline__ int row_param(int off_w, int j, int k) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = k >> 3, jj = (k >> 2) & 1, q = k & 3;
    return off_w + (SL * j + 16 * i + 4 * (lane >> 4) + q) * H + 32 * wave + 16 * jj + (lane & 15);
}

__device__ __forceinline__ RowState load_row_state(const TrainArgs &A, const MemberW &M, int off_w, int j) {
    RowState st;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int off = row_param(off_w, j, k);
        if (A.grad != nullptr) {
            st.w[k] = A.grad[off];
            st.m[k] = st.v[k] = 0.f;
        } else {
            st.w[k] = M.w[off];
            st.m[k] = M.m[off];
            st.v[k] = M.v[off];
        }
    }
    return st;
}

// Weight rows [SL j, SL j + SL) of a 256-wide hidden layer (offset off_w, bias
// off_b): dW[o][i] = sum_r gt[o][r] At[i][r] with gt this workgroup's gradient
// columns (LDS, [SL][GTS]) and At the transposed input activations [H][NB]; then
// the bias rows.  Adam mode writes the new bfloat16 copies into nb (rows) and nt
// (transposed).
__device__ __forceinline__ void wgrad_rows(const TrainArgs &A, const MemberW &M, const AdamC &c, RowState &st,
                                           const uint16_t *gt, const uint16_t *At, int j, int off_w, int off_b,
                                           uint16_t *nb, uint16_t *nt) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n0 = 32 * wave;
    f32x4 acc[2][2];
    zero_acc(acc);
    wave_mma<2, 2, NB, true>(gt, GTS, At + n0 * NB, NB, acc);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            const int in = n0 + 16 * jj + (lane & 15);
            const int o0 = SL * j + 16 * i + 4 * (lane >> 4);
            uint16_t h[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = (2 * i + jj) * 4 + q;
                const int off = off_w + (o0 + q) * H + in;
                if (A.grad != nullptr) {
                    A.grad[off] = st.w[k] + acc[i][jj][q];
                } else {
                    adam_update(st.w[k], st.m[k], st.v[k], acc[i][jj][q], c);
                    M.w[off] = st.w[k];
                    M.m[off] = st.m[k];
                    M.v[off] = st.v[k];
                    h[q] = to_bf16(st.w[k]);
                    nb[(o0 + q) * H + in] = h[q];
                }
            }
            if (A.grad == nullptr) {
                uint2 pk;
                pk.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
                pk.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
                *reinterpret_cast<uint2 *>(nt + in * H + o0) = pk;
            }
        }
    if (threadIdx.x < SL) apply_grad1(A, M, off_b + SL * j + threadIdx.x, row_sum(gt + threadIdx.x * GTS), c);
}

// Layer 1 of a step for columns [SL j, SL j + SL): gathers the step's rows
// (src, LDS) into LDS (xs [NB][X1S]) and forms a, a^T, gelu'(z) with the weight
// rows w1rows ([SL][FP], global or LDS).
__device__ __forceinline__ void forward_first(const TrainArgs &A, const int *src, const uint16_t *w1rows,
                                              const float *b1, int j, unsigned char *sb, uint16_t *xs) {
    for (int e = threadIdx.x; e < NB * FP / 8; e += TRAIN_THREADS) {
        const int r = e / (FP / 8), k8 = (e % (FP / 8)) * 8;
        const int sr = src[r];
        uint4 v = {0u, 0u, 0u, 0u};
        if (sr >= 0) v = *reinterpret_cast<const uint4 *>(A.xn + (long long)sr * FP + k8);
        *reinterpret_cast<uint4 *>(xs + r * X1S + k8) = v;
    }
    __syncthreads();
    fwd_slice<FP>(xs, X1S, w1rows, b1, j, S_A(0), S_AT(0), S_D(0));
}

// Step counters and loss accumulators of a launch sequence start at zero (a
// kernel, not a memset, so the sequence may be captured).
__global__ __launch_bounds__(256) void train_init_kernel(unsigned char *scratch, int members) {
    int *ctr = reinterpret_cast<int *>(scratch);
    if (threadIdx.x < 5) ctr[threadIdx.x] = 0;
    for (int m = threadIdx.x; m < members; m += blockDim.x)
        *reinterpret_cast<double *>(scratch + TS_CTRL + (size_t)m * MEMBER_SCRATCH + MS_LOSS) = 0.0;
}

// Layer 1 of the first step of a sequence (and its rows, for the step's kernels).
__global__ __launch_bounds__(TRAIN_THREADS) void train_f1_kernel(TrainArgs A) {
    __shared__ __attribute__((aligned(16))) uint16_t xs[NB * X1S];
    __shared__ int src[NB];
    const int j = blockIdx.x, mem = A.member + (int)blockIdx.y;
    const MemberW M = member_weights(A.W, mem);
    unsigned char *sb = member_scratch(A);
    const StepPos c = step_pos(A, 0);
    step_rows(A, mem, c, sb, src);
    if (j == 0 && threadIdx.x < NB) reinterpret_cast<int *>(sb + MS_SRC)[threadIdx.x] = src[threadIdx.x];
    forward_first(A, src, M.w1b + SL * j * FP, M.w + OFF_B1, j, sb, xs);
}

// Hidden layer L (2 or 3) of a step.
template <int L>
__global__ __launch_bounds__(TRAIN_THREADS) void train_fwd_kernel(TrainArgs A) {
    const long long g = take_step(A, L == 2 ? K_F2 : K_F3);
    const int j = blockIdx.x, mem = A.member + (int)blockIdx.y;
    const MemberW M = member_weights(A.W, mem);
    const BfView B = bf_view(A.W, mem, A.grad != nullptr ? 0 : (int)(g & 1));
    unsigned char *sb = member_scratch(A);
    fwd_slice<H>(S_A(L - 2), H, (L == 2 ? B.w2b : B.w3b) + SL * j * H, M.w + (L == 2 ? OFF_B2 : OFF_B3), j,
                 S_A(L - 1), S_AT(L - 1), S_D(L - 1));
}

// Output layer, loss, output-layer weight columns, layer-3 gradient and weight rows.
__global__ __launch_bounds__(TRAIN_THREADS) void train_b3_kernel(TrainArgs A) {
    __shared__ __attribute__((aligned(16))) uint16_t g4[NB * G4S];    // [NB][G4S] output gradient
    __shared__ __attribute__((aligned(16))) uint16_t g4t[OP * GTS];   // [OP][GTS]; then layer-3 gradient [SL][GTS]
    __shared__ double s_loss;
    const long long g = take_step(A, K_B3);
    const int j = blockIdx.x, mem = A.member + (int)blockIdx.y;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const MemberW M = member_weights(A.W, mem);
    const bool upd = A.grad == nullptr;
    const int set = upd ? (int)(g & 1) : 0;
    const BfView B = bf_view(A.W, mem, set), N = bf_view(A.W, mem, set ^ 1);
    unsigned char *sb = member_scratch(A);
    RowState st = load_row_state(A, M, OFF_W3, j);
    const StepPos c = step_pos(A, g);
    const AdamC ac = adam_constants(A, c);
    const int *srcs = reinterpret_cast<const int *>(sb + MS_SRC) + (g & 1) * NB;
    if (tid == 0) s_loss = 0.0;
    __syncthreads();
    // ---- output layer over all rows (every workgroup), loss, output gradient
    {
        const int m0 = 32 * wave;
        const float scale = 2.0f / (float)((upd ? (double)c.nbe : (double)A.n) * NO);
        f32x4 acc[2][4];
        zero_acc(acc);
        wave_mma<2, 4, H, true>(S_A(2) + m0 * H, H, B.w4b, H, acc);
        double ls = 0.0;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int row0 = m0 + 16 * i + 4 * (lane >> 4);
            int src[4];
            float t[4][4];
#pragma unroll
            for (int q = 0; q < 4; ++q) src[q] = srcs[row0 + q];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int col = 16 * jj + (lane & 15);
                    t[q][jj] = (col < NO && src[q] >= 0) ? A.tn[(long long)src[q] * NO + col] : 0.f;
                }
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int col = 16 * jj + (lane & 15);
                uint16_t h[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float gv = 0.f;
                    if (col < NO && src[q] >= 0) {
                        const float y = acc[i][jj][q] + M.w[OFF_B4 + col];
                        const float diff = y - t[q][jj];
                        ls += (double)diff * (double)diff;
                        gv = diff * scale;
                    }
                    h[q] = to_bf16(gv);
                    g4[(row0 + q) * G4S + col] = h[q];
                }
                uint2 pk;
                pk.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
                pk.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
                *reinterpret_cast<uint2 *>(g4t + col * GTS + row0) = pk;
            }
        }
        for (int off = 32; off > 0; off >>= 1) ls += __shfl_xor(ls, off);
        if (lane == 0) atomicAdd(&s_loss, ls);
    }
    __syncthreads();
    if (j == 0) {
        if (tid < NO) S_B4G[tid] = row_sum(g4t + tid * GTS);   // applied by the next kernel
        if (tid == 0) {
            double *acc_loss = S_LOSS;
            const double L = *acc_loss + s_loss;
            const bool epoch_end = c.st == c.steps - 1;
            if (upd && epoch_end) {
                if (A.loss_hist != nullptr) A.loss_hist[(size_t)blockIdx.y * A.epochs + c.ep] = (float)(L / ((double)A.n * NO));
                if (A.loss_out != nullptr && blockIdx.y == 0 && c.g == c.total - 1) *A.loss_out = L / ((double)A.n * NO);
                *acc_loss = 0.0;
            } else {
                *acc_loss = L;
                if (!upd && c.g == c.total - 1 && A.loss_out != nullptr) *A.loss_out = L / ((double)A.n * NO);
            }
        }
    }
    // ---- output-layer weight columns [SL j, SL j + SL): dW4[o][i] = sum_r g4t[o][r] A3t[i][r],
    // one 16 x 16 tile per wave (three output tiles, two column tiles)
    if (wave < 6) {
        const int ot = wave % 3, it = wave / 3;
        f32x4 acc[1][1];
        zero_acc(acc);
        wave_mma<1, 1, NB, true>(g4t + 16 * ot * GTS, GTS, S_AT(2) + (SL * j + 16 * it) * NB, NB, acc);
        const int in = SL * j + 16 * it + (lane & 15);
        int off[4];
        float gv[4], w[4];
        bool on[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int o = 16 * ot + 4 * (lane >> 4) + q;
            on[q] = o < NO;
            off[q] = OFF_W4 + min(o, NO - 1) * H + in;
            gv[q] = acc[0][0][q];
        }
        apply_grads<4>(A, M, off, gv, on, ac, w);
        if (upd) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int o = 16 * ot + 4 * (lane >> 4) + q;
                if (o >= NO) continue;
                const uint16_t h = to_bf16(w[q]);
                N.w4b[o * H + in] = h;
                N.w4t[in * OP + o] = h;
            }
        }
    }
    // ---- layer-3 gradient columns (into g4t's memory after the barrier inside)
    bwd_slice<OP>(g4, G4S, B.w4t, S_D(2), j, S_G(0), g4t);
    __syncthreads();
    wgrad_rows(A, M, ac, st, g4t, S_AT(1), j, OFF_W3, OFF_B3, N.w3b, N.w3t);
}

// Output bias, layer-2 gradient and weight rows.
__global__ __launch_bounds__(TRAIN_THREADS) void train_b2_kernel(TrainArgs A) {
    __shared__ __attribute__((aligned(16))) uint16_t gt[SL * GTS];
    const long long g = take_step(A, K_B2);
    const int j = blockIdx.x, mem = A.member + (int)blockIdx.y;
    const MemberW M = member_weights(A.W, mem);
    const bool upd = A.grad == nullptr;
    const int set = upd ? (int)(g & 1) : 0;
    const BfView B = bf_view(A.W, mem, set), N = bf_view(A.W, mem, set ^ 1);
    unsigned char *sb = member_scratch(A);
    RowState st = load_row_state(A, M, OFF_W2, j);
    const StepPos c = step_pos(A, g);
    const AdamC ac = adam_constants(A, c);
    if (j == 0 && threadIdx.x < NO) apply_grad1(A, M, OFF_B4 + threadIdx.x, S_B4G[threadIdx.x], ac);
    bwd_slice<H>(S_G(0), H, B.w3t, S_D(1), j, S_G(1), gt);
    __syncthreads();
    wgrad_rows(A, M, ac, st, gt, S_AT(0), j, OFF_W2, OFF_B2, N.w2b, N.w2t);
}

// Layer-1 gradient and weight rows, then layer 1 of the next step.
__global__ __launch_bounds__(TRAIN_THREADS) void train_b1_kernel(TrainArgs A) {
    __shared__ __attribute__((aligned(16))) uint16_t gt[SL * GTS];
    __shared__ __attribute__((aligned(16))) uint16_t xt[FP * GTS];  // this step's features, transposed
    __shared__ __attribute__((aligned(16))) uint16_t xs[NB * X1S];  // the next step's features
    __shared__ __attribute__((aligned(16))) uint16_t w1s[SL * FP];  // the updated weight rows
    __shared__ int src[NB];
    const long long g = take_step(A, K_B1);
    const int j = blockIdx.x, mem = A.member + (int)blockIdx.y;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const MemberW M = member_weights(A.W, mem);
    const bool upd = A.grad == nullptr;
    const int set = upd ? (int)(g & 1) : 0;
    const BfView B = bf_view(A.W, mem, set), N = bf_view(A.W, mem, set ^ 1);
    unsigned char *sb = member_scratch(A);
    const StepPos c = step_pos(A, g);
    const AdamC ac = adam_constants(A, c);
    const int *srcs = reinterpret_cast<const int *>(sb + MS_SRC) + (g & 1) * NB;
    for (int e = tid; e < NB * FP / 8; e += TRAIN_THREADS) {
        const int r = e / (FP / 8), k8 = (e % (FP / 8)) * 8;
        const int sr = srcs[r];
        uint4 v = {0u, 0u, 0u, 0u};
        if (sr >= 0) v = *reinterpret_cast<const uint4 *>(A.xn + (long long)sr * FP + k8);
        const uint16_t *h = reinterpret_cast<const uint16_t *>(&v);
#pragma unroll
        for (int k = 0; k < 8; ++k) xt[(k8 + k) * GTS + r] = h[k];
    }
    for (int e = tid; e < SL * FP; e += TRAIN_THREADS) w1s[e] = B.w1b[SL * j * FP + e];
    bwd_slice<H>(S_G(1), H, B.w2t, S_D(0), j, nullptr, gt);
    __syncthreads();
    // ---- weight rows of layer 1: dW1[o][k] = sum_r gt[o][r] xt[k][r], k < NF
    if (wave < 2) {
        f32x4 acc[1][1];
        zero_acc(acc);
        wave_mma<1, 1, NB, true>(gt + 16 * wave * GTS, GTS, xt, GTS, acc);
        const int k = lane & 15;
        int off[4];
        float gv[4], w[4];
        bool on[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int o = SL * j + 16 * wave + 4 * (lane >> 4) + q;
            on[q] = k < NF;
            off[q] = OFF_W1 + o * NF + min(k, NF - 1);
            gv[q] = acc[0][0][q];
        }
        apply_grads<4>(A, M, off, gv, on, ac, w);
        if (upd && k < NF) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ol = 16 * wave + 4 * (lane >> 4) + q;
                const uint16_t h = to_bf16(w[q]);
                N.w1b[(SL * j + ol) * FP + k] = h;
                w1s[ol * FP + k] = h;
            }
        }
    }
    if (tid < SL) apply_grad1(A, M, OFF_B1 + SL * j + tid, row_sum(gt + tid * GTS), ac);
    if (g + 1 >= c.total) return;
    // ---- layer 1 of the next step (step_rows begins with a barrier)
    const StepPos cn = step_pos(A, g + 1);
    step_rows(A, mem, cn, sb, src);
    if (j == 0 && tid < NB) reinterpret_cast<int *>(sb + MS_SRC)[((g + 1) & 1) * NB + tid] = src[tid];
    forward_first(A, src, w1s, M.w + OFF_B1, j, sb, xs);
}

// ------------------------------------------------------------------ inference
// One workgroup of four waves takes PT points through every member.  A hidden
// layer's product is split by output columns: wave w forms columns
// [64 w, 64 w + 64) for all PT rows, so each weight is read once per workgroup
// (not once per wave) and used for PT rows; the activations stay in one LDS
// buffer, overwritten in place once every wave has read them.  The output layer
// (36 columns) is split by rows, so each wave holds whole output rows for the
// decode (block norms by lane shuffles).
constexpr int PT = 64;          // points per workgroup
constexpr int XS = FP + 8;      // LDS row strides (bfloat16 elements), padded against bank conflicts
constexpr int HS = H + 8;
constexpr int PTILES = PT / 16;

// GELU of the inference epilogue: z Phi(z) with Phi linearly interpolated in
// the LDS table (interval 16/4096: interpolation error below 5e-7 in Phi, far
// under the bfloat16 rounding the activation takes next; Phi = 0 below -8 and
// 1 above 8 to the same accuracy).  A table lookup and two FMAs replace the
// quarter-rate exponential and reciprocal of the closed form, which made the
// epilogue, not the matrix cores, the bound of the inference kernel.
__device__ __forceinline__ float gelu_lut(float z, const float2 *tab) {
    constexpr float scale = GELU_TAB_N / (2.0f * GELU_TAB_Z);
    const float u = fminf(fmaxf(fmaf(z, scale, GELU_TAB_Z * scale), 0.0f), (float)GELU_TAB_N - 0.5f);
    const int i = (int)u;
    const float2 e = tab[i];
    return z * fmaf(u - (float)i, e.y, e.x);
}

// Phi(z_i) and its increment on each table interval, from the FP64 erfc.
__global__ void gelu_table_kernel(float2 *tab) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= GELU_TAB_N) return;
    const double h = 2.0 * (double)GELU_TAB_Z / GELU_TAB_N;
    const double z0 = -(double)GELU_TAB_Z + h * i, z1 = z0 + h;
    const double p0 = 0.5 * erfc(-z0 * 0.70710678118654752440), p1 = 0.5 * erfc(-z1 * 0.70710678118654752440);
    tab[i] = make_float2((float)p0, (float)(p1 - p0));
}

template <int K>
__device__ __forceinline__ void infer_hidden(const uint16_t *A, int lda, const uint16_t *Wb, const float *bias,
                                             const float2 *tab, uint16_t *out) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n0 = 64 * wave;
    f32x4 acc[PTILES][4];
    zero_acc(acc);
    wave_mma<PTILES, 4, K>(A, lda, Wb + n0 * K, K, acc);
    __syncthreads();   // every wave has read A (out may be A)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = n0 + 16 * j + (lane & 15);
        const float b = bias[col];
#pragma unroll
        for (int i = 0; i < PTILES; ++i) {
            const int row0 = 16 * i + 4 * (lane >> 4);
#pragma unroll
            for (int q = 0; q < 4; ++q) out[(row0 + q) * HS + col] = to_bf16_hw(gelu_lut(acc[i][j][q] + b, tab));
        }
    }
}

__global__ __launch_bounds__(256) void predict_kernel(PredictArgs P) {
    __shared__ __attribute__((aligned(16))) uint16_t xs[PT * XS];
    __shared__ __attribute__((aligned(16))) uint16_t hb[PT * HS];
    __shared__ float s_ymu[NO], s_ysd[NO];
    __shared__ float2 tab[GELU_TAB_N];
    for (int e = threadIdx.x; e < GELU_TAB_N; e += blockDim.x) tab[e] = P.gelu_tab[e];
    static_assert(2 * PT * NO * sizeof(float) <= PT * HS * sizeof(uint16_t), "statistics reuse the activations");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long p0 = (long long)blockIdx.x * PT;
    if (tid < NO) {
        s_ymu[tid] = (float)P.norm[NORM_YMU + tid];
        s_ysd[tid] = (float)P.norm[NORM_YSD + tid];
    }
    if (tid < PT) {
        const long long p = p0 + tid;
        double f[NF];
        bool ok = false;
        if (p < P.n) {
            ok = record_features(P.params + p * 11, P.c_sat, f);
            if (!ok) atomicOr(P.bad, 1);
        }
        for (int k = 0; k < FP; ++k) {
            uint16_t v = 0;
            if (ok && k < NF) v = to_bf16((float)((f[k] - P.norm[NORM_XMU + k]) / P.norm[NORM_XSD + k]));
            xs[tid * XS + k] = v;
        }
    }
    __syncthreads();
    // the output layer's rows of this wave: two row tiles of 16
    constexpr int OT = PTILES / 4;
    float mean[OT][3][4], m2[OT][3][4];
#pragma unroll
    for (int i = 0; i < OT; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) mean[i][j][q] = m2[i][j][q] = 0.f;
#pragma unroll 1
    for (int mem = 0; mem < P.members; ++mem) {
        const MemberW M = member_weights(P.W, mem);
        infer_hidden<FP>(xs, XS, M.w1b, M.w + OFF_B1, tab, hb);
        __syncthreads();
        infer_hidden<H>(hb, HS, M.w2b, M.w + OFF_B2, tab, hb);
        __syncthreads();
        infer_hidden<H>(hb, HS, M.w3b, M.w + OFF_B3, tab, hb);
        __syncthreads();
        {
            f32x4 acc[OT][3];
            zero_acc(acc);
            wave_mma<OT, 3, H>(hb + 16 * OT * wave * HS, HS, M.w4b, H, acc);
            const float cnt = (float)(mem + 1);
            const int c16 = lane & 15, base = lane & ~15;
#pragma unroll
            for (int i = 0; i < OT; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    // decode this row: de-standardise, block norms of the directions
                    // (sums over the 16 lanes holding the row), scale by exp(log-norm)
                    float v[3], s[3] = {0.f, 0.f, 0.f};
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const int col = 16 * j + c16;
                        v[j] = 0.f;
                        if (col < NO) {
                            v[j] = s_ymu[col] + s_ysd[col] * (acc[i][j][q] + M.w[OFF_B4 + col]);
                            if (!col_is_log(col)) s[col_block(col)] += phys_weight(col_phys(col)) * v[j] * v[j];
                        }
                    }
#pragma unroll
                    for (int b = 0; b < 3; ++b)
#pragma unroll
                        for (int off = 8; off > 0; off >>= 1) s[b] += __shfl_xor(s[b], off);
                    const float lnC = __shfl(v[0], base + 0);
                    const float lnK = __shfl(v[1], base + 6);
                    const float lnD = __shfl(v[1], base + 13);
                    const float sc[3] = {expf(lnC) / sqrtf(s[0]), expf(lnK) / sqrtf(s[1]), expf(lnD) / sqrtf(s[2])};
#pragma unroll
                    for (int j = 0; j < 3; ++j) {   // Welford update over members, physical units
                        const int col = 16 * j + c16;
                        const float y = (col < NO && !col_is_log(col)) ? v[j] * sc[col_block(col)] : 0.f;
                        const float dlt = y - mean[i][j][q];
                        mean[i][j][q] += dlt / cnt;
                        m2[i][j][q] += dlt * (y - mean[i][j][q]);
                    }
                }
        }
        __syncthreads();
    }
    // ---- ensemble statistics of each point -> LDS, then one thread per point
    float *smean = reinterpret_cast<float *>(hb);
    float *svar = smean + PT * NO;
#pragma unroll
    for (int i = 0; i < OT; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int col = 16 * j + (lane & 15);
            if (col >= NO) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 16 * (OT * wave + i) + 4 * (lane >> 4) + q;
                smean[row * NO + col] = mean[i][j][q];
                svar[row * NO + col] = P.members > 1 ? m2[i][j][q] / (float)(P.members - 1) : 0.f;
            }
        }
    __syncthreads();
    if (tid < PT) {
        const long long p = p0 + tid;
        if (p < P.n) {
            double y[NPHYS], num[3] = {0, 0, 0}, den[3] = {0, 0, 0};
            for (int col = 0; col < NO; ++col) {
                if (col_is_log(col)) continue;
                const int ph = col_phys(col), blk = col_block(col);
                y[ph] = (double)smean[tid * NO + col];
                const double w = (double)phys_weight(ph);
                num[blk] += w * (double)svar[tid * NO + col];
                den[blk] += w * y[ph] * y[ph];
            }
            double dis = 0.0;
            for (int b = 0; b < 3; ++b) dis = fmax(dis, sqrt(num[b]) / sqrt(den[b]));
            for (int o = 0; o < 21; ++o) P.C[p * 21 + o] = y[o];
            for (int o = 0; o < 6; ++o) {
                P.K[p * 6 + o] = y[21 + o];
                P.D[p * 6 + o] = y[27 + o];
            }
            if (P.dis) P.dis[p] = dis;
        }
    }
}

// ------------------------------------------------------------------ fallback bookkeeping
// List of the points whose disagreement exceeds thresh (or is not finite); the
// order of the list is arbitrary (the host sorts it).
__global__ void select_kernel(const double *dis, long long n, double thresh, int *idx, int *count,
                              unsigned char *flag) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double d = dis[i];
        const bool fb = !(d <= thresh);
        if (flag) flag[i] = fb ? 1 : 0;
        if (fb) {
            const int k = atomicAdd(count, 1);
            idx[k] = (int)i;
        }
    }
}

// Copies records idx[0..m) of params into out (compact).
__global__ void gather_kernel(const double *params, const int *idx, int m, double *out) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m * 11; e += gridDim.x * blockDim.x)
        out[e] = params[(long long)idx[e / 11] * 11 + e % 11];
}

// Writes compact results back to rows idx[0..m) of C, K, D.
__global__ void scatter_kernel(const double *c, const double *k, const double *d, const int *idx, int m, double *C,
                               double *K, double *D) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m * NPHYS; e += gridDim.x * blockDim.x) {
        const int j = e / NPHYS, o = e % NPHYS;
        const long long p = idx[j];
        if (o < 21) C[p * 21 + o] = c[(long long)j * 21 + o];
        else if (o < 27) K[p * 6 + o - 21] = k[(long long)j * 6 + o - 21];
        else D[p * 6 + o - 27] = d[(long long)j * 6 + o - 27];
    }
}

__global__ void fill_kernel(float *p, long long n, float v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

static int grid_of(long long work, int bs) {
    long long g = (work + bs - 1) / bs;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (int)g;
}

// ------------------------------------------------------------------ launchers
hipError_t launch_sync_bf16(const Weights &W, int members, hipStream_t s) {
    const long long per = (long long)H * FP + 2LL * H * H + (long long)OP * H;
    sync_bf16_kernel<<<grid_of(per * members, 256), 256, 0, s>>>(W, members);
    return hipGetLastError();
}

hipError_t launch_stats(const double *params, const double *C, const double *K, const double *D, long long n,
                        double c_sat, double *norm, int *bad, hipStream_t s) {
    stats_kernel<<<NF + NO, 256, 0, s>>>(params, C, K, D, n, c_sat, norm, bad);
    return hipGetLastError();
}

hipError_t launch_prepare(const double *params, const double *C, const double *K, const double *D, long long n,
                          double c_sat, const double *norm, uint16_t *xn, float *tn, int *bad, hipStream_t s) {
    prepare_kernel<<<grid_of(n, 256), 256, 0, s>>>(params, C, K, D, n, c_sat, norm, xn, tn, bad);
    return hipGetLastError();
}

static hipError_t enqueue_train_steps(const TrainArgs &a, dim3 grid, long long steps, hipStream_t s) {
    for (long long i = 0; i < steps; ++i) {
        train_fwd_kernel<2><<<grid, TRAIN_THREADS, 0, s>>>(a);
        train_fwd_kernel<3><<<grid, TRAIN_THREADS, 0, s>>>(a);
        train_b3_kernel<<<grid, TRAIN_THREADS, 0, s>>>(a);
        train_b2_kernel<<<grid, TRAIN_THREADS, 0, s>>>(a);
        train_b1_kernel<<<grid, TRAIN_THREADS, 0, s>>>(a);
    }
    return hipGetLastError();
}

hipError_t launch_train(const TrainArgs &a, int members, hipStream_t s, hipStream_t cap) {
    const dim3 grid(NSL, members);
    const long long total = (a.n + a.nb - 1) / a.nb * (long long)a.epochs;
    train_init_kernel<<<1, 256, 0, s>>>(a.scratch, members);
    train_f1_kernel<<<grid, TRAIN_THREADS, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    constexpr long long G = 64;   // steps per captured graph
    long long done = 0;
    if (cap != nullptr && total >= 2 * G) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        const hipError_t le = enqueue_train_steps(a, grid, G, cap);
        e = hipStreamEndCapture(cap, &graph);
        if (le != hipSuccess) e = le;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        for (; e == hipSuccess && done + G <= total; done += G) e = hipGraphLaunch(exec, s);
        const hipError_t se = hipStreamSynchronize(s);   // the graph is destroyed below
        if (exec != nullptr) (void)hipGraphExecDestroy(exec);
        if (graph != nullptr) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return e;
        if (se != hipSuccess) return se;
    }
    return enqueue_train_steps(a, grid, total - done, s);
}

hipError_t launch_predict(const PredictArgs &a, hipStream_t s) {
    const long long blocks = (a.n + PT - 1) / PT;
    predict_kernel<<<(unsigned)blocks, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_gelu_table(float2 *tab, hipStream_t s) {
    gelu_table_kernel<<<(GELU_TAB_N + 255) / 256, 256, 0, s>>>(tab);
    return hipGetLastError();
}

hipError_t launch_select(const double *dis, long long n, double thresh, int *idx, int *count, unsigned char *flag,
                         hipStream_t s) {
    select_kernel<<<grid_of(n, 256), 256, 0, s>>>(dis, n, thresh, idx, count, flag);
    return hipGetLastError();
}

hipError_t launch_gather(const double *params, const int *idx, int m, double *out, hipStream_t s) {
    gather_kernel<<<grid_of((long long)m * 11, 256), 256, 0, s>>>(params, idx, m, out);
    return hipGetLastError();
}

hipError_t launch_scatter(const double *c, const double *k, const double *d, const int *idx, int m, double *C,
                          double *K, double *D, hipStream_t s) {
    scatter_kernel<<<grid_of((long long)m * NPHYS, 256), 256, 0, s>>>(c, k, d, idx, m, C, K, D);
    return hipGetLastError();
}

hipError_t launch_fill(float *p, long long n, float v, hipStream_t s) {
    fill_kernel<<<grid_of(n, 256), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace chom
