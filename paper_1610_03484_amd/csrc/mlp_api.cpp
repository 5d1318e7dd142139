// C ABI of the learned surrogate: ensemble state, training, prediction and the
// fallback to the RVE solve (kernels in mlp.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "internal.h"
#include "mlp.h"

using namespace chom;
namespace M_ = chom::mlp;

struct chom_mlp {
    chom_mlp_options opt{};
    int members = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    DevBuf<float> master, adam_m, adam_v, grad, loss_hist;
    DevBuf<uint16_t> w1b, w2b, w3b, w4b, w2t, w3t, w4t, alt;
    DevBuf<double> norm, loss;
    bool has_norm = false;
    long long step = 0;           // Adam steps taken (shared by the members)
    long long epochs_done = 0;    // shuffle stream position
    DevBuf<unsigned char> scratch, used;
    DevBuf<uint16_t> xn;
    DevBuf<float> tn;
    DevBuf<double> in_p, in_c, in_k, in_d;         // staging of host inputs
    DevBuf<double> out_c, out_k, out_d, out_dis;   // device results when the caller's are on the host
    DevBuf<double> fb_p, fb_c, fb_k, fb_d;         // compact fallback records / results
    DevBuf<int> flag, idx, count;
    DevBuf<float2> gelu_tab;       // inference GELU table (filled at creation)
    hipStream_t capture = nullptr;   // training graphs are captured here
    ~chom_mlp() {
        if (capture) (void)hipStreamDestroy(capture);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
    M_::Weights weights() const {
        M_::Weights W;
        W.master = master.p;
        W.adam_m = adam_m.p;
        W.adam_v = adam_v.p;
        W.w1b = w1b.p;
        W.w2b = w2b.p;
        W.w3b = w3b.p;
        W.w4b = w4b.p;
        W.w2t = w2t.p;
        W.w3t = w3t.p;
        W.w4t = w4t.p;
        W.alt = alt.p;
        return W;
    }
};

namespace {

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) used counter-style: the state
// is seed * 2^32 + item * 64 + slot; uniform in [0, 1) from the top 53 bits.
double counter_uniform(uint64_t seed, uint64_t item, uint64_t slot) {
    uint64_t z = (seed << 32) + item * 64 + slot + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

void initial_weights(uint64_t seed, int member, std::vector<float> &w) {
    w.assign(M_::NPARAM, 0.0f);
    struct L {
        int off, out, in;
    } layers[4] = {{M_::OFF_W1, M_::H, M_::NF}, {M_::OFF_W2, M_::H, M_::H}, {M_::OFF_W3, M_::H, M_::H},
                   {M_::OFF_W4, M_::NO, M_::H}};
    for (const L &l : layers) {
        const double a = std::sqrt(3.0 / l.in);
        for (int e = 0; e < l.out * l.in; ++e)
            w[l.off + e] = (float)((2.0 * counter_uniform(seed, (uint64_t)(l.off + e), (uint64_t)member) - 1.0) * a);
    }
}

int stage_in(chom_mlp *m, DevBuf<double> &buf, const void *p, size_t count, const double **out) {
    if (m->opt.device_ptrs) {
        *out = static_cast<const double *>(p);
        return CHOM_OK;
    }
    CHOM_HIP(buf.ensure(count));
    CHOM_HIP(hipMemcpyAsync(buf.p, p, sizeof(double) * count, hipMemcpyHostToDevice, m->stream));
    *out = buf.p;
    return CHOM_OK;
}

int check_flag(chom_mlp *m, const char *what) {
    int bad = 0;
    CHOM_HIP(hipMemcpyAsync(&bad, m->flag.p, sizeof(int), hipMemcpyDeviceToHost, m->stream));
    CHOM_HIP(hipStreamSynchronize(m->stream));
    if (bad) {
        set_error(std::string(what) + ": a record is outside the degradation law's domain "
                  "(T >= T_g, negative moisture or time, non-positive factor) or a result is not finite");
        return CHOM_EINVAL;
    }
    return CHOM_OK;
}

// Standardised training rows from n records (inputs already on the device).
int prepare_rows(chom_mlp *m, const double *p, const double *c, const double *k, const double *d, long long n,
                 bool refit, const char *what) {
    CHOM_HIP(m->flag.ensure(1));
    CHOM_HIP(hipMemsetAsync(m->flag.p, 0, sizeof(int), m->stream));
    if (refit) {
        CHOM_HIP(M_::launch_stats(p, c, k, d, n, m->opt.c_sat, m->norm.p, m->flag.p, m->stream));
        m->has_norm = true;
    }
    CHOM_HIP(m->xn.ensure((size_t)n * M_::FP));
    CHOM_HIP(m->tn.ensure((size_t)n * M_::NO));
    CHOM_HIP(M_::launch_prepare(p, c, k, d, n, m->opt.c_sat, m->norm.p, m->xn.p, m->tn.p, m->flag.p, m->stream));
    return check_flag(m, what);
}

int sync_copies(chom_mlp *m) {
    CHOM_HIP(M_::launch_sync_bf16(m->weights(), m->members, m->stream));
    return CHOM_OK;
}

// Predict into device buffers C, K, D, dis (dis nullable).
int predict_device(chom_mlp *m, const double *p, long long n, double *C, double *K, double *D, double *dis) {
    CHOM_HIP(m->flag.ensure(1));
    CHOM_HIP(hipMemsetAsync(m->flag.p, 0, sizeof(int), m->stream));
    M_::PredictArgs a;
    a.gelu_tab = m->gelu_tab.p;
    a.params = p;
    a.n = n;
    a.c_sat = m->opt.c_sat;
    a.norm = m->norm.p;
    a.members = m->members;
    a.W = m->weights();
    a.C = C;
    a.K = K;
    a.D = D;
    a.dis = dis;
    a.bad = m->flag.p;
    CHOM_HIP(M_::launch_predict(a, m->stream));
    return check_flag(m, "chom_mlp_predict");
}

}  // namespace

namespace chom {

// chom_mlp_loss_grad's evaluation on device inputs and outputs, with the rows,
// the flag and the training scratch in the caller's workspace `ws` (layout of
// mlp::ws_bytes(max_rows), 256-byte aligned): no allocation.  All work is queued
// on the handle's stream; returns after the flag has been read back.
int mlp_loss_grad_ws(chom_mlp *m, int member, const double *p, const double *c, const double *k, const double *d,
                     long long n, double *loss, float *grad, unsigned char *ws, long long max_rows) {
    if (n < 1 || n > max_rows) {
        set_error("workspace holds at most " + std::to_string(max_rows) + " records");
        return CHOM_EINVAL;
    }
    int *flag = reinterpret_cast<int *>(ws + M_::WS_FLAG);
    uint16_t *xn = reinterpret_cast<uint16_t *>(ws + M_::WS_XN);
    float *tn = reinterpret_cast<float *>(ws + M_::ws_tn(max_rows));
    unsigned char *tr = ws + M_::ws_train(max_rows);
    // a fill kernel, not a memset, clears the flag (the zero bit pattern)
    CHOM_HIP(M_::launch_fill(reinterpret_cast<float *>(flag), 1, 0.0f, m->stream));
    CHOM_HIP(M_::launch_prepare(p, c, k, d, n, m->opt.c_sat, m->norm.p, xn, tn, flag, m->stream));
    CHOM_HIP(M_::launch_fill(grad, M_::NPARAM, 0.0f, m->stream));
    M_::TrainArgs a;
    std::memset(&a, 0, sizeof(a));
    a.xn = xn;
    a.tn = tn;
    a.n = n;
    a.epochs = 1;
    a.nb = M_::NB;
    a.lr0 = a.lr1 = 0.0f;
    a.beta1 = 0.9f;
    a.beta2 = 0.999f;
    a.eps = 1e-8f;
    a.member = member;
    a.grad = grad;
    a.loss_out = loss;
    a.W = m->weights();
    a.scratch = tr;
    CHOM_HIP(M_::launch_train(a, 1, m->stream, nullptr));
    int bad = 0;
    CHOM_HIP(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, m->stream));
    CHOM_HIP(hipStreamSynchronize(m->stream));
    if (bad) {
        set_error("a record is outside the degradation law's domain or a result is not finite");
        return CHOM_EINVAL;
    }
    return CHOM_OK;
}

bool mlp_ready(const chom_mlp *m, int member) { return m && m->has_norm && member >= 0 && member < m->members; }

int mlp_device_ptrs(const chom_mlp *m) { return m->opt.device_ptrs != 0; }

}  // namespace chom

extern "C" {

int chom_mlp_default_options(chom_mlp_options *opt) {
    if (!opt) return CHOM_EINVAL;
    std::memset(opt, 0, sizeof(*opt));
    opt->members = 5;
    opt->device_ptrs = 0;
    opt->seed = 0;
    opt->c_sat = 1.5;
    opt->hip_stream = nullptr;
    return CHOM_OK;
}

int chom_mlp_default_train_options(chom_mlp_train_options *opt) {
    if (!opt) return CHOM_EINVAL;
    std::memset(opt, 0, sizeof(*opt));
    opt->epochs = 300;
    opt->batch = 256;
    opt->lr = 2e-3f;
    opt->lr_final = 2e-5f;
    opt->beta1 = 0.9f;
    opt->beta2 = 0.999f;
    opt->eps = 1e-8f;
    opt->refit_normalisation = 1;
    return CHOM_OK;
}

int chom_mlp_create(const chom_mlp_options *opt_in, chom_mlp **out) {
    if (!out) {
        set_error("chom_mlp_create: null output handle");
        return CHOM_EINVAL;
    }
    *out = nullptr;
    chom_mlp_options opt;
    if (opt_in) opt = *opt_in;
    else chom_mlp_default_options(&opt);
    if (opt.members < 1 || opt.members > 8 || !(opt.c_sat > 0.0)) {
        set_error("chom_mlp_create: members must be in 1..8 and c_sat positive");
        return CHOM_EINVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        set_error("chom_mlp_create: no HIP device");
        return CHOM_EDEVICE;
    }
    std::unique_ptr<chom_mlp> m(new chom_mlp());
    m->opt = opt;
    m->members = opt.members;
    if (opt.hip_stream) {
        m->stream = (hipStream_t)opt.hip_stream;
    } else {
        CHOM_HIP(hipStreamCreate(&m->stream));
        m->own_stream = true;
    }
    const size_t M = (size_t)opt.members, P = M_::NPARAM;
    CHOM_HIP(m->master.ensure(M * P));
    CHOM_HIP(m->adam_m.ensure(M * P));
    CHOM_HIP(m->adam_v.ensure(M * P));
    CHOM_HIP(m->w1b.ensure(M * M_::H * M_::FP));
    CHOM_HIP(m->w2b.ensure(M * M_::H * M_::H));
    CHOM_HIP(m->w3b.ensure(M * M_::H * M_::H));
    CHOM_HIP(m->w4b.ensure(M * M_::OP * M_::H));
    CHOM_HIP(m->w2t.ensure(M * M_::H * M_::H));
    CHOM_HIP(m->w3t.ensure(M * M_::H * M_::H));
    CHOM_HIP(m->w4t.ensure(M * M_::H * M_::OP));
    CHOM_HIP(m->gelu_tab.ensure(M_::GELU_TAB_N));
    CHOM_HIP(m->norm.ensure(M_::NORM_LEN));
    CHOM_HIP(m->loss.ensure(1));
    CHOM_HIP(m->scratch.ensure((size_t)M_::train_scratch_bytes(M)));
    CHOM_HIP(hipMemsetAsync(m->adam_m.p, 0, sizeof(float) * M * P, m->stream));
    CHOM_HIP(hipMemsetAsync(m->adam_v.p, 0, sizeof(float) * M * P, m->stream));
    std::vector<float> w;
    for (int mem = 0; mem < opt.members; ++mem) {
        initial_weights(opt.seed, mem, w);
        CHOM_HIP(hipMemcpyAsync(m->master.p + (size_t)mem * P, w.data(), sizeof(float) * P, hipMemcpyHostToDevice,
                                m->stream));
        CHOM_HIP(hipStreamSynchronize(m->stream));
    }
    CHOM_TRY(sync_copies(m.get()));
    CHOM_HIP(M_::launch_gelu_table(m->gelu_tab.p, m->stream));
    CHOM_HIP(hipStreamSynchronize(m->stream));
    *out = m.release();
    return CHOM_OK;
}

int chom_mlp_sizes(const chom_mlp *m, int64_t *params_per_member, int32_t *members) {
    if (!m) return CHOM_EINVAL;
    if (params_per_member) *params_per_member = M_::NPARAM;
    if (members) *members = m->members;
    return CHOM_OK;
}

int chom_mlp_set_weights(chom_mlp *m, int32_t member, const float *flat) {
    if (!m || !flat || member < 0 || member >= m->members) {
        set_error("chom_mlp_set_weights: bad handle, member or pointer");
        return CHOM_EINVAL;
    }
    const size_t P = M_::NPARAM;
    for (size_t i = 0; i < P; ++i)
        if (!std::isfinite(flat[i])) {
            set_error("chom_mlp_set_weights: non-finite weight");
            return CHOM_EINVAL;
        }
    CHOM_HIP(hipMemcpyAsync(m->master.p + member * P, flat, sizeof(float) * P, hipMemcpyHostToDevice, m->stream));
    CHOM_HIP(hipMemsetAsync(m->adam_m.p + member * P, 0, sizeof(float) * P, m->stream));
    CHOM_HIP(hipMemsetAsync(m->adam_v.p + member * P, 0, sizeof(float) * P, m->stream));
    m->step = 0;
    CHOM_TRY(sync_copies(m));
    CHOM_HIP(hipStreamSynchronize(m->stream));
    return CHOM_OK;
}

int chom_mlp_get_weights(const chom_mlp *m, int32_t member, float *flat) {
    if (!m || !flat || member < 0 || member >= m->members) {
        set_error("chom_mlp_get_weights: bad handle, member or pointer");
        return CHOM_EINVAL;
    }
    const size_t P = M_::NPARAM;
    CHOM_HIP(hipMemcpyAsync(flat, m->master.p + member * P, sizeof(float) * P, hipMemcpyDeviceToHost, m->stream));
    CHOM_HIP(hipStreamSynchronize(m->stream));
    return CHOM_OK;
}

int chom_mlp_set_normalisation(chom_mlp *m, const double *rec) {
    if (!m || !rec) return CHOM_EINVAL;
    for (int i = 0; i < M_::NORM_LEN; ++i) {
        const bool is_sd = (i >= M_::NORM_XSD && i < M_::NORM_YMU) || i >= M_::NORM_YSD;
        if (!std::isfinite(rec[i]) || (is_sd && !(rec[i] > 0.0))) {
            set_error("chom_mlp_set_normalisation: non-finite entry or non-positive deviation");
            return CHOM_EINVAL;
        }
    }
    CHOM_HIP(hipMemcpyAsync(m->norm.p, rec, sizeof(double) * M_::NORM_LEN, hipMemcpyHostToDevice, m->stream));
    CHOM_HIP(hipStreamSynchronize(m->stream));
    m->has_norm = true;
    return CHOM_OK;
}

int chom_mlp_get_normalisation(const chom_mlp *m, double *rec) {
    if (!m || !rec || !m->has_norm) {
        set_error("chom_mlp_get_normalisation: no standardisation record yet");
        return CHOM_EINVAL;
    }
    CHOM_HIP(hipMemcpyAsync(rec, m->norm.p, sizeof(double) * M_::NORM_LEN, hipMemcpyDeviceToHost, m->stream));
    CHOM_HIP(hipStreamSynchronize(m->stream));
    return CHOM_OK;
}

int chom_mlp_train(chom_mlp *m, const chom_params *params, const double *C, const double *K, const double *D,
                   int64_t n, const chom_mlp_train_options *opt_in, float *loss_history) {
    if (!m || !params || !C || !K || !D || n < 1 || n >= (1LL << 31)) {
        set_error("chom_mlp_train: null argument or n outside [1, 2^31)");
        return CHOM_EINVAL;
    }
    chom_mlp_train_options o;
    if (opt_in) o = *opt_in;
    else chom_mlp_default_train_options(&o);
    if (o.epochs < 1 || o.batch < 1 || o.batch > M_::NB || !(o.lr > 0.0f) || !(o.lr_final >= 0.0f) ||
        !(o.beta1 >= 0.0f && o.beta1 < 1.0f) || !(o.beta2 >= 0.0f && o.beta2 < 1.0f) || !(o.eps > 0.0f)) {
        set_error("chom_mlp_train: epochs >= 1, batch in 1..256, lr > 0, betas in [0, 1), eps > 0 required");
        return CHOM_EINVAL;
    }
    const double *p, *c, *k, *d;
    CHOM_TRY(stage_in(m, m->in_p, params, (size_t)n * 11, &p));
    CHOM_TRY(stage_in(m, m->in_c, C, (size_t)n * 21, &c));
    CHOM_TRY(stage_in(m, m->in_k, K, (size_t)n * 6, &k));
    CHOM_TRY(stage_in(m, m->in_d, D, (size_t)n * 6, &d));
    CHOM_TRY(prepare_rows(m, p, c, k, d, n, o.refit_normalisation != 0 || !m->has_norm, "chom_mlp_train"));
    CHOM_HIP(m->loss_hist.ensure((size_t)m->members * o.epochs));
    // second set of bfloat16 copies (steps alternate between the sets); the
    // padding rows and columns, which no step writes, stay zero
    CHOM_HIP(m->alt.ensure((size_t)m->members * M_::BF_PER_MEMBER));
    CHOM_HIP(hipMemsetAsync(m->alt.p, 0, sizeof(uint16_t) * m->alt.n, m->stream));
    if (m->capture == nullptr) CHOM_HIP(hipStreamCreateWithFlags(&m->capture, hipStreamNonBlocking));
    M_::TrainArgs a;
    std::memset(&a, 0, sizeof(a));
    a.xn = m->xn.p;
    a.tn = m->tn.p;
    a.n = n;
    a.epochs = o.epochs;
    a.epoch0 = (int)m->epochs_done;
    a.nb = o.batch;
    a.lr0 = o.lr;
    a.lr1 = o.lr_final;
    a.beta1 = o.beta1;
    a.beta2 = o.beta2;
    a.eps = o.eps;
    a.seed = m->opt.seed;
    a.step0 = m->step;
    a.member = 0;
    a.grad = nullptr;
    a.loss_hist = m->loss_hist.p;
    a.loss_out = m->loss.p;
    a.W = m->weights();
    a.scratch = m->scratch.p;
    CHOM_HIP(M_::launch_train(a, m->members, m->stream, m->capture));
    CHOM_TRY(sync_copies(m));   // the last step's copies may be in the second set
    CHOM_HIP(hipStreamSynchronize(m->stream));
    m->step += ((n + o.batch - 1) / o.batch) * (long long)o.epochs;
    m->epochs_done += o.epochs;
    if (loss_history)
        CHOM_HIP(hipMemcpy(loss_history, m->loss_hist.p, sizeof(float) * (size_t)m->members * o.epochs,
                           hipMemcpyDeviceToHost));
    return CHOM_OK;
}

int chom_mlp_loss_grad(chom_mlp *m, int32_t member, const chom_params *params, const double *C, const double *K,
                       const double *D, int64_t n, double *loss, float *grad) {
    if (!m || !params || !C || !K || !D || !loss || !grad || n < 1 || n >= (1LL << 31) || member < 0 ||
        member >= m->members) {
        set_error("chom_mlp_loss_grad: bad argument");
        return CHOM_EINVAL;
    }
    if (!m->has_norm) {
        set_error("chom_mlp_loss_grad: no standardisation record (set one or train first)");
        return CHOM_EINVAL;
    }
    const double *p, *c, *k, *d;
    CHOM_TRY(stage_in(m, m->in_p, params, (size_t)n * 11, &p));
    CHOM_TRY(stage_in(m, m->in_c, C, (size_t)n * 21, &c));
    CHOM_TRY(stage_in(m, m->in_k, K, (size_t)n * 6, &k));
    CHOM_TRY(stage_in(m, m->in_d, D, (size_t)n * 6, &d));
    CHOM_TRY(prepare_rows(m, p, c, k, d, n, false, "chom_mlp_loss_grad"));
    CHOM_HIP(m->grad.ensure(M_::NPARAM));
    CHOM_HIP(M_::launch_fill(m->grad.p, M_::NPARAM, 0.0f, m->stream));
    M_::TrainArgs a;
    std::memset(&a, 0, sizeof(a));
    a.xn = m->xn.p;
    a.tn = m->tn.p;
    a.n = n;
    a.epochs = 1;
    a.nb = M_::NB;
    a.lr0 = a.lr1 = 0.0f;
    a.beta1 = 0.9f;
    a.beta2 = 0.999f;
    a.eps = 1e-8f;
    a.member = member;
    a.grad = m->grad.p;
    a.loss_out = m->loss.p;
    a.W = m->weights();
    a.scratch = m->scratch.p;
    CHOM_HIP(M_::launch_train(a, 1, m->stream, nullptr));
    CHOM_HIP(hipMemcpyAsync(grad, m->grad.p, sizeof(float) * M_::NPARAM, hipMemcpyDeviceToHost, m->stream));
    CHOM_HIP(hipMemcpyAsync(loss, m->loss.p, sizeof(double), hipMemcpyDeviceToHost, m->stream));
    CHOM_HIP(hipStreamSynchronize(m->stream));
    return CHOM_OK;
}

int chom_mlp_predict(chom_mlp *m, const chom_params *params, int64_t n, double *C, double *K, double *D,
                     double *dis) {
    if (!m || !params || !C || !K || !D || n < 1 || n >= (1LL << 40)) {
        set_error("chom_mlp_predict: bad argument");
        return CHOM_EINVAL;
    }
    if (!m->has_norm) {
        set_error("chom_mlp_predict: no standardisation record (set one or train first)");
        return CHOM_EINVAL;
    }
    const double *p;
    CHOM_TRY(stage_in(m, m->in_p, params, (size_t)n * 11, &p));
    if (m->opt.device_ptrs) return predict_device(m, p, n, C, K, D, dis);
    CHOM_HIP(m->out_c.ensure((size_t)n * 21));
    CHOM_HIP(m->out_k.ensure((size_t)n * 6));
    CHOM_HIP(m->out_d.ensure((size_t)n * 6));
    CHOM_HIP(m->out_dis.ensure((size_t)n));
    CHOM_TRY(predict_device(m, p, n, m->out_c.p, m->out_k.p, m->out_d.p, dis ? m->out_dis.p : nullptr));
    CHOM_HIP(hipMemcpyAsync(C, m->out_c.p, sizeof(double) * n * 21, hipMemcpyDeviceToHost, m->stream));
    CHOM_HIP(hipMemcpyAsync(K, m->out_k.p, sizeof(double) * n * 6, hipMemcpyDeviceToHost, m->stream));
    CHOM_HIP(hipMemcpyAsync(D, m->out_d.p, sizeof(double) * n * 6, hipMemcpyDeviceToHost, m->stream));
    if (dis) CHOM_HIP(hipMemcpyAsync(dis, m->out_dis.p, sizeof(double) * n, hipMemcpyDeviceToHost, m->stream));
    CHOM_HIP(hipStreamSynchronize(m->stream));
    return CHOM_OK;
}

int chom_homogenise_surrogate(chom_mlp *m, chom_rve *fallback, const chom_params *params, int64_t n,
                              double thresh, int32_t chunk, double *C, double *K, double *D, double *dis_out,
                              uint8_t *used_fallback, int64_t *n_fallback) {
    if (!m || !fallback || !params || !C || !K || !D || n < 1 || n >= (1LL << 31) || chunk < 0 ||
        !(thresh >= 0.0)) {
        set_error("chom_homogenise_surrogate: bad argument");
        return CHOM_EINVAL;
    }
    if (m->members < 2) {
        set_error("chom_homogenise_surrogate: the disagreement needs at least two members");
        return CHOM_EINVAL;
    }
    if (!m->has_norm) {
        set_error("chom_homogenise_surrogate: the ensemble is not trained (no standardisation record)");
        return CHOM_EINVAL;
    }
    double rc = 0.0;
    int ry = 0;
    rve_settings(fallback, &rc, &ry);
    if (rc != m->opt.c_sat) {
        set_error("chom_homogenise_surrogate: the RVE and the ensemble use different c_sat");
        return CHOM_EINVAL;
    }
    const bool dev = m->opt.device_ptrs != 0;
    const double *p;
    CHOM_TRY(stage_in(m, m->in_p, params, (size_t)n * 11, &p));
    double *dc = C, *dk = K, *dd = D;
    if (!dev) {
        CHOM_HIP(m->out_c.ensure((size_t)n * 21));
        CHOM_HIP(m->out_k.ensure((size_t)n * 6));
        CHOM_HIP(m->out_d.ensure((size_t)n * 6));
        dc = m->out_c.p;
        dk = m->out_k.p;
        dd = m->out_d.p;
    }
    double *ddis = (dev && dis_out) ? dis_out : nullptr;
    if (!ddis) {
        CHOM_HIP(m->out_dis.ensure((size_t)n));
        ddis = m->out_dis.p;
    }
    unsigned char *dused = (dev && used_fallback) ? used_fallback : nullptr;
    if (!dused) {
        CHOM_HIP(m->used.ensure((size_t)n));
        dused = m->used.p;
    }
    CHOM_TRY(predict_device(m, p, n, dc, dk, dd, ddis));
    CHOM_HIP(m->idx.ensure((size_t)n));
    CHOM_HIP(m->count.ensure(1));
    CHOM_HIP(hipMemsetAsync(m->count.p, 0, sizeof(int), m->stream));
    CHOM_HIP(M_::launch_select(ddis, n, thresh, m->idx.p, m->count.p, dused, m->stream));
    int cnt = 0;
    CHOM_HIP(hipMemcpyAsync(&cnt, m->count.p, sizeof(int), hipMemcpyDeviceToHost, m->stream));
    CHOM_HIP(hipStreamSynchronize(m->stream));
    int status = CHOM_OK;
    if (cnt > 0) {
        std::vector<int> hidx(cnt);
        CHOM_HIP(hipMemcpy(hidx.data(), m->idx.p, sizeof(int) * cnt, hipMemcpyDeviceToHost));
        std::sort(hidx.begin(), hidx.end());
        CHOM_HIP(hipMemcpy(m->idx.p, hidx.data(), sizeof(int) * cnt, hipMemcpyHostToDevice));
        CHOM_HIP(m->fb_p.ensure((size_t)cnt * 11));
        CHOM_HIP(M_::launch_gather(p, m->idx.p, cnt, m->fb_p.p, m->stream));
        std::vector<chom_params> hp(cnt);
        CHOM_HIP(hipMemcpyAsync(hp.data(), m->fb_p.p, sizeof(double) * cnt * 11, hipMemcpyDeviceToHost, m->stream));
        CHOM_HIP(hipStreamSynchronize(m->stream));
        const int cs = std::min(cnt, chunk > 0 ? chunk : 256);
        std::vector<double> rc_((size_t)cnt * 21), rk((size_t)cnt * 6), rd((size_t)cnt * 6);
        std::vector<chom_params> cp(cs);
        std::vector<double> tc((size_t)cs * 21), tk((size_t)cs * 6), td((size_t)cs * 6);
        for (int s0 = 0; s0 < cnt; s0 += cs) {
            const int mcount = std::min(cs, cnt - s0);
            for (int j = 0; j < cs; ++j) cp[j] = hp[s0 + std::min(j, mcount - 1)];   // pad with a real record
            const int st = rve_homogenise_host(fallback, cp.data(), cs, tc.data(), tk.data(), td.data(), nullptr);
            if (st == CHOM_ENOCONV) status = CHOM_ENOCONV;
            else if (st != CHOM_OK) return st;
            std::copy(tc.begin(), tc.begin() + (size_t)mcount * 21, rc_.begin() + (size_t)s0 * 21);
            std::copy(tk.begin(), tk.begin() + (size_t)mcount * 6, rk.begin() + (size_t)s0 * 6);
            std::copy(td.begin(), td.begin() + (size_t)mcount * 6, rd.begin() + (size_t)s0 * 6);
        }
        CHOM_HIP(m->fb_c.ensure((size_t)cnt * 21));
        CHOM_HIP(m->fb_k.ensure((size_t)cnt * 6));
        CHOM_HIP(m->fb_d.ensure((size_t)cnt * 6));
        CHOM_HIP(hipMemcpyAsync(m->fb_c.p, rc_.data(), sizeof(double) * rc_.size(), hipMemcpyHostToDevice, m->stream));
        CHOM_HIP(hipMemcpyAsync(m->fb_k.p, rk.data(), sizeof(double) * rk.size(), hipMemcpyHostToDevice, m->stream));
        CHOM_HIP(hipMemcpyAsync(m->fb_d.p, rd.data(), sizeof(double) * rd.size(), hipMemcpyHostToDevice, m->stream));
        CHOM_HIP(M_::launch_scatter(m->fb_c.p, m->fb_k.p, m->fb_d.p, m->idx.p, cnt, dc, dk, dd, m->stream));
    }
    if (!dev) {
        CHOM_HIP(hipMemcpyAsync(C, dc, sizeof(double) * n * 21, hipMemcpyDeviceToHost, m->stream));
        CHOM_HIP(hipMemcpyAsync(K, dk, sizeof(double) * n * 6, hipMemcpyDeviceToHost, m->stream));
        CHOM_HIP(hipMemcpyAsync(D, dd, sizeof(double) * n * 6, hipMemcpyDeviceToHost, m->stream));
        if (dis_out) CHOM_HIP(hipMemcpyAsync(dis_out, ddis, sizeof(double) * n, hipMemcpyDeviceToHost, m->stream));
        if (used_fallback)
            CHOM_HIP(hipMemcpyAsync(used_fallback, dused, (size_t)n, hipMemcpyDeviceToHost, m->stream));
    }
    CHOM_HIP(hipStreamSynchronize(m->stream));
    if (n_fallback) *n_fallback = cnt;
    if (status != CHOM_OK) set_error("chom_homogenise_surrogate: some fallback load case did not converge");
    return status;
}

void chom_mlp_destroy(chom_mlp *m) { delete m; }

}  // extern "C"
