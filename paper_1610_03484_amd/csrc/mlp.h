// Shapes, layouts and launchers of the surrogate network kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chom {
namespace mlp {

constexpr int NF = 10;            // features: log(1 - omega), (1 - omega), 8 factors
constexpr int FP = 32;            // features padded to one MFMA contraction step
constexpr int H = 256;            // hidden width
constexpr int NO = 36;            // network outputs: per block (C 21, K 6, D 6) log-norm + direction
constexpr int NPHYS = 33;         // physical outputs: C upper 21, K 6, D 6
constexpr int OP = 64;            // outputs padded (contraction of the first backward product)
constexpr int NB = 256;           // largest minibatch
constexpr int TRAIN_THREADS = 512;   // eight waves
constexpr int SL = 32;            // hidden columns per training workgroup
constexpr int NSL = H / SL;       // training workgroups per member

// Flat FP32 parameter layout of one member (row-major [out][in] matrices).
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + H * NF;
constexpr int OFF_W2 = OFF_B1 + H;
constexpr int OFF_B2 = OFF_W2 + H * H;
constexpr int OFF_W3 = OFF_B2 + H;
constexpr int OFF_B3 = OFF_W3 + H * H;
constexpr int OFF_W4 = OFF_B3 + H;
constexpr int OFF_B4 = OFF_W4 + NO * H;
constexpr int NPARAM = OFF_B4 + NO;   // 143,652

// Standardisation record (FP64): feature means, feature deviations, encoded-output means and deviations.
constexpr int NORM_XMU = 0;
constexpr int NORM_XSD = NF;
constexpr int NORM_YMU = 2 * NF;
constexpr int NORM_YSD = 2 * NF + NO;
constexpr int NORM_LEN = 2 * NF + 2 * NO;

// Training scratch: a control block (the step counters of a launch sequence),
// then per member the minibatch arrays shared by its workgroups (byte offsets):
// activations of the three hidden layers row-major and transposed (bfloat16),
// gelu'(z) (FP32), the hidden gradients of layers 3 and 2 (bfloat16), the
// output-bias gradient of the step, the minibatch rows, the epoch's shuffle and
// the loss accumulator.
constexpr long long TS_CTRL = 256;
constexpr long long MS_A = 0;
constexpr long long MS_AT = MS_A + 3LL * NB * H * 2;
constexpr long long MS_D = MS_AT + 3LL * NB * H * 2;
constexpr long long MS_G = MS_D + 3LL * NB * H * 4;
constexpr long long MS_B4G = MS_G + 2LL * NB * H * 2;
constexpr long long MS_SRC = MS_B4G + 256;          // 2 x [NB] source rows of a step (by step parity)
constexpr long long MS_PERM = MS_SRC + 2LL * NB * 4;  // the current epoch's shuffle (2 x int64)
constexpr long long MS_LOSS = MS_PERM + 16;
constexpr long long MEMBER_SCRATCH = MS_LOSS + 240;
constexpr long long train_scratch_bytes(int members) { return TS_CTRL + members * MEMBER_SCRATCH; }

// bfloat16 copies of one member's weights (elements): w1b [H][FP], w2b, w3b
// [H][H], w4b [OP][H], w2t, w3t [H][H], w4t [H][OP].
constexpr long long BF_PER_MEMBER = (long long)H * FP + 4LL * H * H + 2LL * OP * H;

// Workspace of a gradient evaluation in caller-provided memory (no allocation):
// the bad-record flag, the standardised rows of up to `rows` records (bfloat16
// features, FP32 targets) and the training scratch of one member, each part
// 256-byte aligned.
constexpr long long ws_align(long long b) { return (b + 255) / 256 * 256; }
constexpr long long WS_FLAG = 0;
constexpr long long WS_XN = 256;
constexpr long long ws_tn(long long rows) { return WS_XN + ws_align(rows * FP * 2); }
constexpr long long ws_train(long long rows) { return ws_tn(rows) + ws_align(rows * NO * 4); }
constexpr long long ws_bytes(long long rows) { return ws_train(rows) + ws_align(train_scratch_bytes(1)); }

// Degradation law of Sec. 4 (constant exposure).
constexpr double BETA = -0.001682;    // per day
constexpr double TG_CELSIUS = 126.0;
constexpr double KELVIN = 273.15;
constexpr double DAYS_PER_YEAR = 365.25;

struct Weights {                 // all members, member-major
    float *master, *adam_m, *adam_v;            // [M][NPARAM]
    uint16_t *w1b, *w2b, *w3b, *w4b;            // bfloat16 copies [M][H][FP], [M][H][H] x2, [M][OP][H]
    uint16_t *w2t, *w3t, *w4t;                  // transposes [M][H][H] x2, [M][H][OP]
    uint16_t *alt;                              // training: second set of copies, [M][BF_PER_MEMBER]
};

struct TrainArgs {
    const uint16_t *xn;          // [n][FP] standardised features (bfloat16)
    const float *tn;             // [n][NO] standardised targets
    long long n;
    int epochs, epoch0, nb;      // epoch0: index of the first epoch (shuffle stream)
    float lr0, lr1, beta1, beta2, eps;
    unsigned long long seed;
    long long step0;             // Adam steps taken before this launch sequence
    int member;                  // first member (gradient mode: the member)
    float *grad;                 // gradient mode: accumulate dLoss/dparam here (NPARAM), no update
    float *loss_hist;            // [members][epochs] or null
    double *loss_out;            // loss of the last epoch (or of the gradient evaluation)
    Weights W;
    unsigned char *scratch;      // train_scratch_bytes(members)
};

// Inference GELU table: the standard normal distribution function Phi on
// GELU_TAB_N equal intervals of [-GELU_TAB_Z, GELU_TAB_Z], as (Phi(z_i),
// Phi(z_{i+1}) - Phi(z_i)) pairs.
constexpr int GELU_TAB_N = 4096;
constexpr float GELU_TAB_Z = 8.0f;

struct PredictArgs {
    const float2 *gelu_tab;      // GELU_TAB_N entries (launch_gelu_table)
    const double *params;        // [n][11]
    long long n;
    double c_sat;
    const double *norm;          // NORM_LEN
    int members;
    Weights W;
    double *C, *K, *D, *dis;     // outputs [n][21], [n][6], [n][6], [n] (dis nullable)
    int *bad;
};

hipError_t launch_sync_bf16(const Weights &W, int members, hipStream_t s);
hipError_t launch_stats(const double *params, const double *C, const double *K, const double *D, long long n,
                        double c_sat, double *norm, int *bad, hipStream_t s);
hipError_t launch_prepare(const double *params, const double *C, const double *K, const double *D, long long n,
                          double c_sat, const double *norm, uint16_t *xn, float *tn, int *bad, hipStream_t s);
// Training (or, with a.grad set, gradient accumulation) over a.epochs epochs of
// minibatches, `members` members at once.  Every step is five kernels; `cap` is
// an optional stream on which the library captures a HIP graph of up to 64 steps
// that it then replays on s (null: the kernels are launched one by one).
hipError_t launch_train(const TrainArgs &a, int members, hipStream_t s, hipStream_t cap);
hipError_t launch_predict(const PredictArgs &a, hipStream_t s);
hipError_t launch_gelu_table(float2 *tab, hipStream_t s);
hipError_t launch_select(const double *dis, long long n, double thresh, int *idx, int *count, unsigned char *flag,
                         hipStream_t s);
hipError_t launch_gather(const double *params, const int *idx, int m, double *out, hipStream_t s);
hipError_t launch_scatter(const double *c, const double *k, const double *d, const int *idx, int m, double *C,
                          double *K, double *D, hipStream_t s);
hipError_t launch_fill(float *p, long long n, float v, hipStream_t s);

}  // namespace mlp
}  // namespace chom
