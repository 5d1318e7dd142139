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
constexpr int TRAIN_THREADS = 512;

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

// Minibatch scratch of one training workgroup (bytes).
constexpr long long SCRATCH_BYTES = 2LL * NB * FP * 2 + (long long)NB * NO * 4 + 6LL * NB * H * 2 +
                                    3LL * NB * H * 4 + 2LL * NB * OP * 2 + 6LL * NB * H * 2;

// Workspace of a gradient evaluation in caller-provided memory (no allocation):
// the bad-record flag, the standardised rows of up to `rows` records (bfloat16
// features, FP32 targets) and one training workgroup's minibatch scratch, each
// part 256-byte aligned.
constexpr long long ws_align(long long b) { return (b + 255) / 256 * 256; }
constexpr long long WS_FLAG = 0;
constexpr long long WS_XN = 256;
constexpr long long ws_tn(long long rows) { return WS_XN + ws_align(rows * FP * 2); }
constexpr long long ws_train(long long rows) { return ws_tn(rows) + ws_align(rows * NO * 4); }
constexpr long long ws_bytes(long long rows) { return ws_train(rows) + ws_align(SCRATCH_BYTES); }

// Degradation law of Sec. 4 (constant exposure).
constexpr double BETA = -0.001682;    // per day
constexpr double TG_CELSIUS = 126.0;
constexpr double KELVIN = 273.15;
constexpr double DAYS_PER_YEAR = 365.25;

struct Weights {                 // all members, member-major
    float *master, *adam_m, *adam_v;            // [M][NPARAM]
    uint16_t *w1b, *w2b, *w3b, *w4b;            // bfloat16 copies [M][H][FP], [M][H][H] x2, [M][OP][H]
    uint16_t *w2t, *w3t, *w4t;                  // transposes [M][H][H] x2, [M][H][OP]
};

struct TrainArgs {
    const uint16_t *xn;          // [n][FP] standardised features (bfloat16)
    const float *tn;             // [n][NO] standardised targets
    long long n;
    int epochs, epoch0, nb;      // epoch0: index of the first epoch (shuffle stream)
    float lr0, lr1, beta1, beta2, eps;
    unsigned long long seed;
    long long step0;             // Adam steps taken before this launch
    int member;                  // first member (gradient mode: the member)
    float *grad;                 // gradient mode: accumulate dLoss/dparam here (NPARAM), no update
    float *loss_hist;            // [members][epochs] or null
    double *loss_out;            // loss of the last epoch (or of the gradient evaluation)
    Weights W;
    unsigned char *scratch;      // members x SCRATCH_BYTES
};

struct PredictArgs {
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
hipError_t launch_train(const TrainArgs &a, int blocks, hipStream_t s);
hipError_t launch_predict(const PredictArgs &a, hipStream_t s);
hipError_t launch_select(const double *dis, long long n, double thresh, int *idx, int *count, unsigned char *flag,
                         hipStream_t s);
hipError_t launch_gather(const double *params, const int *idx, int m, double *out, hipStream_t s);
hipError_t launch_scatter(const double *c, const double *k, const double *d, const int *idx, int m, double *C,
                          double *K, double *D, hipStream_t s);
hipError_t launch_fill(float *p, long long n, float v, hipStream_t s);

}  // namespace mlp
}  // namespace chom
