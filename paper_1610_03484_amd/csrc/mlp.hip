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
// Training: one workgroup per ensemble member runs every epoch and minibatch
// (forward, backward, Adam) in one launch; members never exchange data, so the
// launch needs no grid-wide synchronisation.  Activations of the minibatch live
// in a per-member global scratch (L2 resident); each is stored row-major for
// the next layer's product and transposed for the weight-gradient product, so
// that both operands of every product are contiguous along the contraction.
//
// Inference: one workgroup per 128 points evaluates every member with the
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

// The phases of a training step are separate (non-inlined) functions: inlined
// into the step loop, the compiler hoists every phase's loop-invariant address
// arithmetic out of the loop at once and spills.
//
// One wave: acc[i][j] += A[16i.., :K] * B[16j.., :K]^T for 16x16 tiles; A and B are
// bfloat16, row-major with the contraction index contiguous (row strides lda, ldb).
// Lane l supplies row (l & 15) and the 8 contraction entries starting at 8 (l >> 4)
// of each operand tile; the result element (4 (l >> 4) + q, l & 15) of tile (i, j)
// lands in acc[i][j][q].
template <int TM, int TN, int K>
__device__ __forceinline__ void wave_mma(const uint16_t *__restrict__ A, int lda, const uint16_t *__restrict__ B,
                                         int ldb, f32x4 (&acc)[TM][TN]) {
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, kq = (lane >> 4) << 3;
    const uint16_t *Ap = A + r * lda + kq;
    const uint16_t *Bp = B + r * ldb + kq;
#pragma unroll 2
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

// Minibatch scratch of one member (SCRATCH_BYTES): byte offsets of each array.
constexpr long long SO_XB = 0;                                   // [NB][FP] bf16
constexpr long long SO_XBT = SO_XB + NB * FP * 2;                // [FP][NB] bf16
constexpr long long SO_TB = SO_XBT + NB * FP * 2;                // [NB][NO] f32
constexpr long long SO_A = SO_TB + NB * NO * 4;                  // 3 x [NB][H] bf16 (hidden outputs)
constexpr long long SO_AT = SO_A + 3LL * NB * H * 2;             // 3 x [H][NB] bf16 (transposed)
constexpr long long SO_D = SO_AT + 3LL * NB * H * 2;             // 3 x [NB][H] f32 (gelu'(z))
constexpr long long SO_G4 = SO_D + 3LL * NB * H * 4;             // [NB][OP] bf16 (output gradient)
constexpr long long SO_G4T = SO_G4 + NB * OP * 2;                // [OP][NB] bf16
constexpr long long SO_G = SO_G4T + NB * OP * 2;                 // 3 x [NB][H] bf16 (hidden gradients)
constexpr long long SO_GT = SO_G + 3LL * NB * H * 2;             // 3 x [H][NB] bf16
static_assert(SO_GT + 3LL * NB * H * 2 == SCRATCH_BYTES, "scratch layout");

template <typename T> __device__ __forceinline__ T *sp(unsigned char *base, long long off) {
    return reinterpret_cast<T *>(base + off);
}
#define S_XB sp<uint16_t>(sb, SO_XB)
#define S_XBT sp<uint16_t>(sb, SO_XBT)
#define S_TB sp<float>(sb, SO_TB)
#define S_A(l) sp<uint16_t>(sb, SO_A + (l) * (long long)NB * H * 2)
#define S_AT(l) sp<uint16_t>(sb, SO_AT + (l) * (long long)NB * H * 2)
#define S_D(l) sp<float>(sb, SO_D + (l) * (long long)NB * H * 4)
#define S_G4 sp<uint16_t>(sb, SO_G4)
#define S_G4T sp<uint16_t>(sb, SO_G4T)
#define S_G(l) sp<uint16_t>(sb, SO_G + (l) * (long long)NB * H * 2)
#define S_GT(l) sp<uint16_t>(sb, SO_GT + (l) * (long long)NB * H * 2)

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
struct AdamC {
    float lr, b1, b2, eps, bc1, bc2;
};

__device__ __forceinline__ float adam_update(float *w, float *m, float *v, float g, const AdamC &c) {
    const float mm = c.b1 * *m + (1.0f - c.b1) * g;
    const float vv = c.b2 * *v + (1.0f - c.b2) * g * g;
    *m = mm;
    *v = vv;
    const float nw = *w - c.lr * (mm / c.bc1) / (sqrtf(vv / c.bc2) + c.eps);
    *w = nw;
    return nw;
}

// Hidden layer forward over the NB minibatch rows: z = A W^T + b, a = gelu(z).
// Writes a (row-major and transposed, bfloat16) and gelu'(z) (FP32).
template <int K>
__device__ __noinline__ void fwd_hidden(const uint16_t *A, const uint16_t *Wb, const float *bias, uint16_t *aout,
                                           uint16_t *atout, float *dout) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = 32 * wave;
#pragma unroll 1
    for (int ch = 0; ch < 4; ++ch) {
        const int n0 = 64 * ch;
        f32x4 acc[2][4];
        zero_acc(acc);
        wave_mma<2, 4, K>(A + m0 * K, K, Wb + n0 * K, K, acc);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int col = n0 + 16 * j + (lane & 15);
                const int row0 = m0 + 16 * i + 4 * (lane >> 4);
                const float b = bias[col];
                uint16_t h[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float z = acc[i][j][q] + b;
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

// Backward through a hidden layer's input: g = bf16((G Wt^T) * gelu'(z)), with G
// [NB][K] and Wt [H][K] (the transpose of the layer's weights).  Writes g
// row-major (when grow) and transposed.
template <int K>
__device__ __noinline__ void bwd_data(const uint16_t *G, const uint16_t *Wt, const float *dprev, uint16_t *grow,
                                         uint16_t *gtr) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = 32 * wave;
#pragma unroll 1
    for (int ch = 0; ch < 4; ++ch) {
        const int n0 = 64 * ch;
        f32x4 acc[2][4];
        zero_acc(acc);
        wave_mma<2, 4, K>(G + m0 * K, K, Wt + n0 * K, K, acc);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int col = n0 + 16 * j + (lane & 15);
                const int row0 = m0 + 16 * i + 4 * (lane >> 4);
                uint16_t h[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    h[q] = to_bf16(acc[i][j][q] * dprev[(row0 + q) * H + col]);
                    if (grow) grow[(row0 + q) * H + col] = h[q];
                }
                uint2 pk;
                pk.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
                pk.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
                *reinterpret_cast<uint2 *>(gtr + col * NB + row0) = pk;
            }
    }
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

// Gradient of one weight entry: accumulate (gradient mode) or Adam-update the master
// and return the new value through *nw.
__device__ __forceinline__ bool apply_grad(const MemberW &M, float *grad, int off, float g, const AdamC &c,
                                           float *nw) {
    if (grad) {
        grad[off] += g;
        return false;
    }
    *nw = adam_update(M.w + off, M.m + off, M.v + off, g, c);
    return true;
}

// Weight gradient of a 256 x 256 layer (l = 2 or 3): dW[o][i] = sum_r Gt[o][r] At[i][r].
__device__ __noinline__ void wgrad_hidden(const MemberW &M, float *grad, const uint16_t *Gt, const uint16_t *At,
                                             int off_w, uint16_t *wb, uint16_t *wt, const AdamC &c) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = 32 * wave;
#pragma unroll 1
    for (int ch = 0; ch < 4; ++ch) {
        const int n0 = 64 * ch;
        f32x4 acc[2][4];
        zero_acc(acc);
        wave_mma<2, 4, NB>(Gt + m0 * NB, NB, At + n0 * NB, NB, acc);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int in = n0 + 16 * j + (lane & 15);
                const int o0 = m0 + 16 * i + 4 * (lane >> 4);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float nw;
                    if (apply_grad(M, grad, off_w + (o0 + q) * H + in, acc[i][j][q], c, &nw)) {
                        const uint16_t h = to_bf16(nw);
                        wb[(o0 + q) * H + in] = h;
                        wt[in * H + o0 + q] = h;
                    }
                }
            }
    }
}

// Weight gradient of the output layer: dW4[o][i] = sum_r G4t[o][r] A3t[i][r], o < NO.
__device__ __noinline__ void wgrad_out(const MemberW &M, float *grad, const uint16_t *G4t, const uint16_t *A3t,
                                          const AdamC &c) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // 3 row tiles (rows 48..63 are padding) x 4 column quarters = 12 jobs over 8 waves
#pragma unroll 1
    for (int job = wave; job < 12; job += TRAIN_THREADS / 64) {
        const int o_tile = job % 3, quarter = job / 3;
        f32x4 acc[1][4];
        zero_acc(acc);
        wave_mma<1, 4, NB>(G4t + 16 * o_tile * NB, NB, A3t + 64 * quarter * NB, NB, acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int in = 64 * quarter + 16 * j + (lane & 15);
            const int o0 = 16 * o_tile + 4 * (lane >> 4);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int o = o0 + q;
                if (o >= NO) continue;
                float nw;
                if (apply_grad(M, grad, OFF_W4 + o * H + in, acc[0][j][q], c, &nw)) {
                    const uint16_t h = to_bf16(nw);
                    M.w4b[o * H + in] = h;
                    M.w4t[in * OP + o] = h;
                }
            }
        }
    }
}

// Weight gradient of the first layer: dW1[o][k] = sum_r G1t[o][r] Xt[k][r], k < NF.
__device__ __noinline__ void wgrad_first(const MemberW &M, float *grad, const uint16_t *G1t, const uint16_t *Xt,
                                            const AdamC &c) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = 32 * wave;
    f32x4 acc[2][1];
    zero_acc(acc);
    wave_mma<2, 1, NB>(G1t + m0 * NB, NB, Xt, NB, acc);
    const int k = lane & 15;
    if (k >= NF) return;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int o0 = m0 + 16 * i + 4 * (lane >> 4);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float nw;
            if (apply_grad(M, grad, OFF_W1 + (o0 + q) * NF + k, acc[i][0][q], c, &nw))
                M.w1b[(o0 + q) * FP + k] = to_bf16(nw);
        }
    }
}

__device__ __noinline__ void bias_grad(const MemberW &M, float *grad, const uint16_t *gt_row, int off, const AdamC &c) {
    const float g = row_sum(gt_row);
    float nw;
    (void)apply_grad(M, grad, off, g, c, &nw);
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

// One minibatch step of one member: gather, forward, loss, backward, update.
__device__ __noinline__ void train_step(const TrainArgs &A, const MemberW &M, unsigned char *sb, long long st,
                                        long long total, long long gstep, long long pa, long long pb,
                                        double *s_loss) {
    const int tid = threadIdx.x, lane = tid & 63;
    const long long n = A.n;
    const int nb = A.nb;
    const long long i0 = st * nb;
    const int nbe = (int)min((long long)nb, n - i0);
    // ---- gather the minibatch (rows past nbe are zero): one shuffled row index per thread
    __shared__ int s_src[NB];
    if (tid < NB) s_src[tid] = tid < nbe ? (int)perm_index(i0 + tid, n, pa, pb) : -1;
    __syncthreads();
    for (int e = tid; e < NB * FP; e += TRAIN_THREADS) {
        const int r = e / FP, k = e - (e / FP) * FP;
        const int src = s_src[r];
        const uint16_t v = src >= 0 ? A.xn[(long long)src * FP + k] : (uint16_t)0;
        S_XB[r * FP + k] = v;
        S_XBT[k * NB + r] = v;
    }
    for (int e = tid; e < NB * NO; e += TRAIN_THREADS) {
        const int r = e / NO, o = e - (e / NO) * NO;
        const int src = s_src[r];
        S_TB[e] = src >= 0 ? A.tn[(long long)src * NO + o] : 0.f;
    }
    __syncthreads();
    // ---- forward
    fwd_hidden<FP>(S_XB, M.w1b, M.w + OFF_B1, S_A(0), S_AT(0), S_D(0));
    __syncthreads();
    fwd_hidden<H>(S_A(0), M.w2b, M.w + OFF_B2, S_A(1), S_AT(1), S_D(1));
    __syncthreads();
    fwd_hidden<H>(S_A(1), M.w3b, M.w + OFF_B3, S_A(2), S_AT(2), S_D(2));
    __syncthreads();
    // ---- output layer, loss and output gradient
    {
        const int wave = tid >> 6;
        const int m0 = 32 * wave;
        const float scale = 2.0f / (float)((A.grad != nullptr ? (double)n : (double)nbe) * NO);
        f32x4 acc[2][4];
        zero_acc(acc);
        wave_mma<2, 4, H>(S_A(2) + m0 * H, H, M.w4b, H, acc);
        double ls = 0.0;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int col = 16 * j + (lane & 15);
                const int row0 = m0 + 16 * i + 4 * (lane >> 4);
                uint16_t h[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float g = 0.f;
                    if (col < NO && row0 + q < nbe) {
                        const float y = acc[i][j][q] + M.w[OFF_B4 + col];
                        const float diff = y - S_TB[(row0 + q) * NO + col];
                        ls += (double)diff * (double)diff;
                        g = diff * scale;
                    }
                    h[q] = to_bf16(g);
                    S_G4[(row0 + q) * OP + col] = h[q];
                }
                uint2 pk;
                pk.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
                pk.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
                *reinterpret_cast<uint2 *>(S_G4T + col * NB + row0) = pk;
            }
        for (int off = 32; off > 0; off >>= 1) ls += __shfl_xor(ls, off);
        if (lane == 0) atomicAdd(s_loss, ls);
    }
    __syncthreads();
    // ---- backward
    AdamC c;
    {
        const long long t = A.step0 + gstep + 1;
        const double frac = total > 1 ? (double)gstep / (double)(total - 1) : 1.0;
        const double lr = A.lr1 + 0.5 * (A.lr0 - A.lr1) * (1.0 + cos(3.14159265358979323846 * frac));
        c.lr = (float)lr;
        c.b1 = A.beta1;
        c.b2 = A.beta2;
        c.eps = A.eps;
        c.bc1 = (float)(1.0 - pow((double)A.beta1, (double)t));
        c.bc2 = (float)(1.0 - pow((double)A.beta2, (double)t));
    }
    bwd_data<OP>(S_G4, M.w4t, S_D(2), S_G(2), S_GT(2));
    __syncthreads();
    wgrad_out(M, A.grad, S_G4T, S_AT(2), c);
    if (tid < NO) bias_grad(M, A.grad, S_G4T + tid * NB, OFF_B4 + tid, c);
    bwd_data<H>(S_G(2), M.w3t, S_D(1), S_G(1), S_GT(1));
    __syncthreads();
    wgrad_hidden(M, A.grad, S_GT(2), S_AT(1), OFF_W3, M.w3b, M.w3t, c);
    if (tid < H) bias_grad(M, A.grad, S_GT(2) + tid * NB, OFF_B3 + tid, c);
    bwd_data<H>(S_G(1), M.w2t, S_D(0), nullptr, S_GT(0));
    __syncthreads();
    wgrad_hidden(M, A.grad, S_GT(1), S_AT(0), OFF_W2, M.w2b, M.w2t, c);
    wgrad_first(M, A.grad, S_GT(0), S_XBT, c);
    if (tid < H) bias_grad(M, A.grad, S_GT(1) + tid * NB, OFF_B2 + tid, c);
    else bias_grad(M, A.grad, S_GT(0) + (tid - H) * NB, OFF_B1 + (tid - H), c);
    __syncthreads();
}

__global__ __launch_bounds__(TRAIN_THREADS) void train_kernel(TrainArgs A) {
    const int mem = A.grad != nullptr ? A.member : A.member + (int)blockIdx.x;
    const MemberW M = member_weights(A.W, mem);
    unsigned char *sb = A.scratch + (A.grad != nullptr ? 0 : (size_t)blockIdx.x * SCRATCH_BYTES);
    const int tid = threadIdx.x;
    __shared__ double s_loss;
    __shared__ long long s_pa, s_pb;
    const long long n = A.n;
    const long long steps = (n + A.nb - 1) / A.nb;
    const long long total = steps * (long long)A.epochs;
    long long gstep = 0;
    if (tid == 0) s_loss = 0.0;
    for (int ep = 0; ep < A.epochs; ++ep) {
        if (tid == 0) {
            if (A.grad != nullptr || n == 1) {
                s_pa = 1;
                s_pb = 0;
            } else {
                const uint64_t key = (A.seed << 32) + ((uint64_t)mem << 20) + (uint64_t)(A.epoch0 + ep);
                long long a = 1 + (long long)(splitmix(key) % (uint64_t)(n - 1));
                while (gcd_ll(a, n) != 1) a = a % (n - 1) + 1;      // ends: a = 1 is coprime
                s_pa = a;
                s_pb = (long long)(splitmix(key ^ 0x5DEECE66Dull) % (uint64_t)n);
            }
            if (A.grad == nullptr) s_loss = 0.0;
        }
        __syncthreads();
        const long long pa = s_pa, pb = s_pb;
        for (long long st = 0; st < steps; ++st, ++gstep) {
            train_step(A, M, sb, st, total, gstep, pa, pb, &s_loss);
        }
        if (tid == 0 && A.loss_hist != nullptr && A.grad == nullptr)
            A.loss_hist[(size_t)(mem - A.member) * A.epochs + ep] = (float)(s_loss / ((double)n * NO));
    }
    if (tid == 0 && A.loss_out != nullptr) *A.loss_out = s_loss / ((double)n * NO);
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

template <int K>
__device__ __forceinline__ void infer_hidden(const uint16_t *A, int lda, const uint16_t *Wb, const float *bias,
                                             uint16_t *out) {
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
            for (int q = 0; q < 4; ++q) out[(row0 + q) * HS + col] = to_bf16_hw(gelu(acc[i][j][q] + b));
        }
    }
}

__global__ __launch_bounds__(256) void predict_kernel(PredictArgs P) {
    __shared__ __attribute__((aligned(16))) uint16_t xs[PT * XS];
    __shared__ __attribute__((aligned(16))) uint16_t hb[PT * HS];
    __shared__ float s_ymu[NO], s_ysd[NO];
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
        infer_hidden<FP>(xs, XS, M.w1b, M.w + OFF_B1, hb);
        __syncthreads();
        infer_hidden<H>(hb, HS, M.w2b, M.w + OFF_B2, hb);
        __syncthreads();
        infer_hidden<H>(hb, HS, M.w3b, M.w + OFF_B3, hb);
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

hipError_t launch_train(const TrainArgs &a, int blocks, hipStream_t s) {
    train_kernel<<<blocks, TRAIN_THREADS, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_predict(const PredictArgs &a, hipStream_t s) {
    const long long blocks = (a.n + PT - 1) / PT;
    predict_kernel<<<(unsigned)blocks, 256, 0, s>>>(a);
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
