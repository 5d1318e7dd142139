// Time history of the matrix damage at many macro Gauss points (paper Sec. 4,
// Eq. Eq_Model_RateForm): d(1 - omega)/dt = -gamma(c) alpha(T) (1 - omega),
// alpha(T) = beta ln(1 - T/T_g) with absolute temperatures (Eq. Eq_alphaT),
// gamma(c) = c / c_sat (Eq. Eq_Model3), stepped with implicit (backward) Euler as
// the paper states:
//   (1 - omega)_k = (1 - omega)_{k-1} / (1 + gamma(c_k) alpha(T_k) dt_k).
// One thread per point walks its steps; the history arrays are step-major, so a
// wave reads one step of 64 consecutive points in one coalesced access.  The
// kernel streams 16 B in (T, c) and 8 B out per point and step: HBM-bound.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace chom {
namespace {

constexpr double kBeta = -0.001682;   // per day (Sec. 4, Eq. Eq_alphaT_LSF)
constexpr double kTgK = 126.0 + 273.15;
constexpr double kKelvin = 273.15;
constexpr double kDaysPerYear = 365.25;
constexpr double kTrefC = 60.0;       // temperature of the equivalent constant exposure

__global__ __launch_bounds__(256) void damage_history_kernel(long long n, int m, const double *__restrict__ T,
                                                             const double *__restrict__ c,
                                                             const double *__restrict__ dt_years,
                                                             const double *__restrict__ keep0, double inv_csat,
                                                             double *__restrict__ keep, double *__restrict__ last,
                                                             int *bad) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double w = keep0 != nullptr ? keep0[i] : 1.0;
    bool ok = w > 0.0 && w <= 1.0;
    for (int k = 0; k < m; ++k) {
        const long long o = (long long)k * n + i;
        const double Tk = T[o], ck = c[o], dt = dt_years[k];
        const double arg = 1.0 - (Tk + kKelvin) / kTgK;
        ok = ok && arg > 0.0 && ck >= 0.0 && dt >= 0.0;
        const double rate = (ck * inv_csat) * (kBeta * log(arg));   // per day
        w = w / (1.0 + rate * (dt * kDaysPerYear));
        if (keep != nullptr) keep[o] = w;
    }
    if (last != nullptr) last[i] = w;
    if (!ok || !(w > 0.0)) atomicOr(bad, 1);
}

// Equivalent constant-exposure records: T = 60 C, c = c_sat, the time after which
// Eq. Eq_Model_final1 gives the final factor, and the point's property factors.
__global__ __launch_bounds__(256) void equivalent_params_kernel(long long n, const double *__restrict__ last,
                                                                const double *__restrict__ factors, double c_sat,
                                                                double *__restrict__ params) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double alpha_ref = kBeta * log(1.0 - (kTrefC + kKelvin) / kTgK);
    double *p = params + i * 11;
    p[0] = kTrefC;
    p[1] = c_sat;
    p[2] = -log(last[i]) / (alpha_ref * kDaysPerYear);
    for (int f = 0; f < 8; ++f) p[3 + f] = factors != nullptr ? factors[i * 8 + f] : 1.0;
}

unsigned grid_for(long long n) { return (unsigned)((n + 255) / 256); }

// Host or device input: the device pointer to read (staging host data into `buf`).
int stage(bool dev, const double *p, size_t count, DevBuf<double> &buf, hipStream_t s, const double **out) {
    if (p == nullptr || dev) {
        *out = p;
        return CHOM_OK;
    }
    CHOM_HIP(buf.ensure(count));
    CHOM_HIP(hipMemcpyAsync(buf.p, p, sizeof(double) * count, hipMemcpyHostToDevice, s));
    *out = buf.p;
    return CHOM_OK;
}

}  // namespace
}  // namespace chom

using namespace chom;

extern "C" int chom_damage_history(int64_t n, int32_t m, const double *T_celsius, const double *c_wt,
                                   const double *dt_years, const double *keep0, const double *factors,
                                   double c_sat, int32_t device_ptrs, void *hip_stream, double *keep,
                                   chom_params *params_out) {
    if (n < 1 || m < 1 || !T_celsius || !c_wt || !dt_years || (!keep && !params_out) || !(c_sat > 0.0) ||
        n > (1LL << 40) || (long long)n * m > (1LL << 40)) {
        set_error("chom_damage_history: need n, m >= 1, histories, dt, c_sat > 0 and an output");
        return CHOM_EINVAL;
    }
    const bool dev = device_ptrs != 0;
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t nm = (size_t)n * (size_t)m;
    DevBuf<double> bT, bc, bdt, bk0, bf, bkeep, blast, bpar;
    DevBuf<int> bbad;
    const double *dT, *dc, *ddt, *dk0, *df;
    CHOM_TRY(stage(dev, T_celsius, nm, bT, s, &dT));
    CHOM_TRY(stage(dev, c_wt, nm, bc, s, &dc));
    CHOM_TRY(stage(dev, dt_years, (size_t)m, bdt, s, &ddt));
    CHOM_TRY(stage(dev, keep0, (size_t)n, bk0, s, &dk0));
    CHOM_TRY(stage(dev, factors, (size_t)n * 8, bf, s, &df));
    double *dkeep = nullptr;
    if (keep) {
        if (dev) {
            dkeep = keep;
        } else {
            CHOM_HIP(bkeep.ensure(nm));
            dkeep = bkeep.p;
        }
    }
    double *dlast = nullptr, *dpar = nullptr;
    if (params_out) {
        CHOM_HIP(blast.ensure((size_t)n));
        dlast = blast.p;
        if (dev) {
            dpar = reinterpret_cast<double *>(params_out);
        } else {
            CHOM_HIP(bpar.ensure((size_t)n * 11));
            dpar = bpar.p;
        }
    }
    CHOM_HIP(bbad.ensure(1));
    CHOM_HIP(hipMemsetAsync(bbad.p, 0, sizeof(int), s));
    damage_history_kernel<<<grid_for(n), 256, 0, s>>>(n, m, dT, dc, ddt, dk0, 1.0 / c_sat, dkeep, dlast, bbad.p);
    CHOM_HIP(hipGetLastError());
    if (params_out) {
        equivalent_params_kernel<<<grid_for(n), 256, 0, s>>>(n, dlast, df, c_sat, dpar);
        CHOM_HIP(hipGetLastError());
    }
    int hbad = 0;
    CHOM_HIP(hipMemcpyAsync(&hbad, bbad.p, sizeof(int), hipMemcpyDeviceToHost, s));
    if (!dev) {
        if (keep) CHOM_HIP(hipMemcpyAsync(keep, dkeep, sizeof(double) * nm, hipMemcpyDeviceToHost, s));
        if (params_out) CHOM_HIP(hipMemcpyAsync(params_out, dpar, sizeof(double) * n * 11, hipMemcpyDeviceToHost, s));
    }
    CHOM_HIP(hipStreamSynchronize(s));
    if (hbad) {
        set_error("chom_damage_history: exposure outside the law's domain (T >= T_g, c < 0, dt < 0, keep0 not in "
                  "(0, 1]) or a factor underflowed to zero");
        return CHOM_EINVAL;
    }
    return CHOM_OK;
}
