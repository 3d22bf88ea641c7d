// C ABI of the differentiable test-particle tracking: a handle that owns the
// device buffers, a forward call that keeps the checkpoints, and a backward
// call that turns them into the gradient of the final polarization.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/spinpic.h"
#include "track.h"

using namespace spinpic;

namespace {

thread_local std::string g_track_error;

std::string fmt(const char* f, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, f);
    vsnprintf(buf, sizeof buf, f, ap);
    va_end(ap);
    return buf;
}

}  // namespace

struct pic_track {
    pic_track_config cfg{};
    long long n = 0;
    int nseg = 0;
    size_t rsize = 0;             // bytes per value: 4 (FP32) or 8 (FP64)
    pic_allocator alloc{};
    bool has_alloc = false;
    hipStream_t stream = nullptr;
    std::vector<void*> live;
    void *state0 = nullptr, *fin = nullptr, *ckpt = nullptr, *scratch = nullptr, *grad = nullptr;
    double* gte = nullptr;        // per-particle parameter derivatives, 2 x n
    double* acc = nullptr;        // 8 doubles of sums
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    float ms[2] = {0.f, 0.f};
    bool have_forward = false;
    double E0 = 0.0, kp = 0.0;
    std::string err;

    void* dalloc(size_t bytes) {
        void* p = nullptr;
        if (has_alloc) p = alloc.alloc(alloc.user, bytes ? bytes : 256);
        else if (hipMalloc(&p, bytes ? bytes : 256) != hipSuccess) p = nullptr;
        if (p) live.push_back(p);
        return p;
    }
    void release() {
        if (stream || !live.empty()) (void)hipStreamSynchronize(stream);
        for (void* p : live) {
            if (has_alloc) alloc.free(alloc.user, p);
            else (void)hipFree(p);
        }
        live.clear();
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    int fail(int code, const std::string& msg) {
        err = msg;
        return code;
    }
    template <typename real>
    TrackParams<real> params() const {
        TrackParams<real> P;
        const double r = cfg.Z / cfg.mu;
        P.E0 = (real)E0;
        P.kp = (real)kp;
        P.dt = (real)cfg.dt;
        P.half_dt = (real)(0.5 * cfg.dt);
        P.r = (real)r;
        P.a = (real)cfg.a;
        P.eps = (real)(0.5 * r * cfg.dt);
        P.nsteps = cfg.nsteps;
        P.K = cfg.checkpoint;
        return P;
    }
};

#define TRY_HIP(tr, expr)                                                                  \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess) return (tr)->fail(PIC_EHIP, fmt("%s: %s", #expr, hipGetErrorString(_e))); \
    } while (0)

namespace {

// rows (n x 3, three arrays) -> SoA values of the handle's precision
template <typename real>
void pack(const double* x, const double* u, const double* s, long long n, std::vector<unsigned char>& out) {
    out.resize((size_t)9 * n * sizeof(real));
    real* v = reinterpret_cast<real*>(out.data());
    const double* src[3] = {x, u, s};
    for (int q = 0; q < 3; ++q)
        for (int c = 0; c < 3; ++c)
            for (long long i = 0; i < n; ++i) v[(size_t)(3 * q + c) * n + i] = (real)src[q][3 * i + c];
}

template <typename real>
void unpack(const std::vector<unsigned char>& in, long long n, double* x, double* u, double* s) {
    const real* v = reinterpret_cast<const real*>(in.data());
    double* dst[3] = {x, u, s};
    for (int q = 0; q < 3; ++q) {
        if (!dst[q]) continue;
        for (int c = 0; c < 3; ++c)
            for (long long i = 0; i < n; ++i) dst[q][3 * i + c] = (double)v[(size_t)(3 * q + c) * n + i];
    }
}

bool all_finite(const double* a, long long m) {
    for (long long i = 0; i < m; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

}  // namespace

extern "C" {

int pic_track_create(const pic_track_config* cfg, int64_t n, const pic_allocator* alloc, void* hip_stream,
                     pic_track** out) {
    g_track_error.clear();
    if (!out) {
        g_track_error = "out is NULL";
        return PIC_EINVAL;
    }
    *out = nullptr;
    if (!cfg) {
        g_track_error = "cfg is NULL";
        return PIC_EINVAL;
    }
    const pic_track_config& c = *cfg;
    if (n < 1 || n > (1LL << 31)) {
        g_track_error = fmt("n = %lld outside 1..2^31", (long long)n);
        return PIC_EINVAL;
    }
    if (!(c.mu > 0.0) || !std::isfinite(c.mu) || !std::isfinite(c.Z) || !std::isfinite(c.a)) {
        g_track_error = "species: mass must be positive, Z and a finite";
        return PIC_EINVAL;
    }
    if (!(c.dt > 0.0) || !std::isfinite(c.dt)) {
        g_track_error = "dt must be positive and finite";
        return PIC_EINVAL;
    }
    if (c.nsteps < 0 || c.checkpoint < 1) {
        g_track_error = fmt("need nsteps >= 0 and checkpoint >= 1 (got %d, %d)", c.nsteps, c.checkpoint);
        return PIC_EINVAL;
    }
    if (c.precision != PIC_FP64 && c.precision != PIC_FP32_MIXED) {
        g_track_error = fmt("unknown precision %d", c.precision);
        return PIC_EINVAL;
    }
    if (alloc && (!alloc->alloc || !alloc->free)) {
        g_track_error = "allocator needs both alloc and free";
        return PIC_EINVAL;
    }
    pic_track* tr = new pic_track();
    tr->cfg = c;
    tr->n = n;
    tr->stream = (hipStream_t)hip_stream;
    if (alloc) {
        tr->alloc = *alloc;
        tr->has_alloc = true;
    }
    tr->rsize = c.precision == PIC_FP64 ? 8 : 4;
    const int K = std::min(c.checkpoint, std::max(c.nsteps, 1));
    tr->cfg.checkpoint = K;
    tr->nseg = (c.nsteps + K - 1) / K;
    const size_t state = (size_t)9 * n * tr->rsize;
    tr->state0 = tr->dalloc(state);
    tr->fin = tr->dalloc((size_t)9 * n * sizeof(double));
    tr->grad = tr->dalloc(state);
    tr->ckpt = tr->dalloc(state * (size_t)std::max(tr->nseg, 1));
    tr->scratch = tr->dalloc(state * (size_t)K);
    tr->gte = (double*)tr->dalloc((size_t)2 * n * sizeof(double));
    tr->acc = (double*)tr->dalloc(8 * sizeof(double));
    bool ok = tr->state0 && tr->fin && tr->grad && tr->ckpt && tr->scratch && tr->gte && tr->acc;
    for (auto& e : tr->ev) ok = ok && hipEventCreate(&e) == hipSuccess;
    if (!ok) {
        g_track_error = fmt("device allocation for %lld particles failed", (long long)n);
        tr->release();
        delete tr;
        return PIC_ENOMEM;
    }
    *out = tr;
    return PIC_OK;
}

int pic_track_forward(pic_track* tr, double E0, double kp, const double* x0, const double* u0,
                      const double* s0, double P_out[3], double* x_out, double* u_out, double* s_out) {
    if (!tr) return PIC_ESTATE;
    if (!x0 || !u0 || !s0 || !P_out) return tr->fail(PIC_EINVAL, "x0, u0, s0 and P_out must not be NULL");
    if (!std::isfinite(E0) || !std::isfinite(kp)) return tr->fail(PIC_EINVAL, "E0 and kp must be finite");
    const long long n = tr->n;
    if (!all_finite(x0, 3 * n) || !all_finite(u0, 3 * n) || !all_finite(s0, 3 * n))
        return tr->fail(PIC_EINVAL, "initial state holds a non-finite value");
    tr->have_forward = false;
    tr->E0 = E0;
    tr->kp = kp;
    std::vector<unsigned char> h;
    const bool f64 = tr->rsize == 8;
    if (f64) pack<double>(x0, u0, s0, n, h);
    else pack<float>(x0, u0, s0, n, h);
    TRY_HIP(tr, hipMemcpyAsync(tr->state0, h.data(), h.size(), hipMemcpyHostToDevice, tr->stream));
    TRY_HIP(tr, hipMemsetAsync(tr->acc, 0, 8 * sizeof(double), tr->stream));
    TRY_HIP(tr, hipEventRecord(tr->ev[0], tr->stream));
    if (f64)
        TRY_HIP(tr, launch_track_forward<double>(tr->params<double>(), n, (const double*)tr->state0,
                                                 (double*)tr->ckpt, (double*)tr->fin, tr->acc, tr->stream));
    else
        TRY_HIP(tr, launch_track_forward<float>(tr->params<float>(), n, (const float*)tr->state0,
                                                (float*)tr->ckpt, (double*)tr->fin, tr->acc, tr->stream));
    TRY_HIP(tr, hipEventRecord(tr->ev[1], tr->stream));
    double acc[8];
    TRY_HIP(tr, hipMemcpyAsync(acc, tr->acc, sizeof acc, hipMemcpyDeviceToHost, tr->stream));
    std::vector<unsigned char> fin;
    if (x_out || u_out || s_out) {
        fin.resize((size_t)9 * n * sizeof(double));
        TRY_HIP(tr, hipMemcpyAsync(fin.data(), tr->fin, fin.size(), hipMemcpyDeviceToHost, tr->stream));
    }
    TRY_HIP(tr, hipStreamSynchronize(tr->stream));
    TRY_HIP(tr, hipEventElapsedTime(&tr->ms[0], tr->ev[0], tr->ev[1]));
    for (int k = 0; k < 3; ++k) P_out[k] = acc[k] / (double)n;
    if (x_out || u_out || s_out) unpack<double>(fin, n, x_out, u_out, s_out);
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(P_out[k])) return tr->fail(PIC_ENONFINITE, "final polarization is not finite");
    tr->have_forward = true;
    return PIC_OK;
}

int pic_track_backward(pic_track* tr, const double c[3], double grad_theta[2], double* grad_x0,
                       double* grad_u0, double* grad_s0, double* grad_theta_each) {
    if (!tr) return PIC_ESTATE;
    if (!tr->have_forward) return tr->fail(PIC_ESTATE, "no forward run to differentiate");
    if (!c || !grad_theta) return tr->fail(PIC_EINVAL, "c and grad_theta must not be NULL");
    if (!all_finite(c, 3)) return tr->fail(PIC_EINVAL, "c must be finite");
    const long long n = tr->n;
    const bool f64 = tr->rsize == 8;
    TRY_HIP(tr, hipMemsetAsync(tr->acc, 0, 8 * sizeof(double), tr->stream));
    TRY_HIP(tr, hipEventRecord(tr->ev[2], tr->stream));
    if (f64)
        TRY_HIP(tr, launch_track_backward<double>(tr->params<double>(), n, (const double*)tr->state0,
                                                  (const double*)tr->ckpt,
                                                  (double*)tr->scratch, c, (double*)tr->grad,
                                                  grad_theta_each ? tr->gte : nullptr, tr->acc, tr->stream));
    else
        TRY_HIP(tr, launch_track_backward<float>(tr->params<float>(), n, (const float*)tr->state0,
                                                 (const float*)tr->ckpt,
                                                 (float*)tr->scratch, c, (float*)tr->grad,
                                                 grad_theta_each ? tr->gte : nullptr, tr->acc, tr->stream));
    TRY_HIP(tr, hipEventRecord(tr->ev[3], tr->stream));
    double acc[8];
    TRY_HIP(tr, hipMemcpyAsync(acc, tr->acc, sizeof acc, hipMemcpyDeviceToHost, tr->stream));
    std::vector<unsigned char> h;
    if (grad_x0 || grad_u0 || grad_s0) {
        h.resize((size_t)9 * n * tr->rsize);
        TRY_HIP(tr, hipMemcpyAsync(h.data(), tr->grad, h.size(), hipMemcpyDeviceToHost, tr->stream));
    }
    std::vector<double> g2;
    if (grad_theta_each) {
        g2.resize((size_t)2 * n);
        TRY_HIP(tr, hipMemcpyAsync(g2.data(), tr->gte, g2.size() * sizeof(double), hipMemcpyDeviceToHost,
                                   tr->stream));
    }
    TRY_HIP(tr, hipStreamSynchronize(tr->stream));
    TRY_HIP(tr, hipEventElapsedTime(&tr->ms[1], tr->ev[2], tr->ev[3]));
    grad_theta[0] = acc[0];
    grad_theta[1] = acc[1];
    if (!h.empty()) {
        if (f64) unpack<double>(h, n, grad_x0, grad_u0, grad_s0);
        else unpack<float>(h, n, grad_x0, grad_u0, grad_s0);
    }
    if (grad_theta_each)
        for (long long i = 0; i < n; ++i) {
            grad_theta_each[2 * i] = g2[i];
            grad_theta_each[2 * i + 1] = g2[n + i];
        }
    if (!std::isfinite(grad_theta[0]) || !std::isfinite(grad_theta[1]))
        return tr->fail(PIC_ENONFINITE, "gradient is not finite");
    return PIC_OK;
}

int pic_track_timing(pic_track* tr, double ms_out[2]) {
    if (!tr) return PIC_ESTATE;
    if (!ms_out) return tr->fail(PIC_EINVAL, "ms_out must not be NULL");
    ms_out[0] = tr->ms[0];
    ms_out[1] = tr->ms[1];
    return PIC_OK;
}

const char* pic_track_last_error(const pic_track* tr) {
    return tr ? tr->err.c_str() : g_track_error.c_str();
}

void pic_track_free(pic_track* tr) {
    if (!tr) return;
    tr->release();
    delete tr;
}

}  // extern "C"
