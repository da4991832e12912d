// lbml_abi.cpp -- extern "C" entry points of the learned initialiser
// (declared in include/lbml.h): workspace layout, forward / backward / Adam
// sequencing of the kernels in lbml_kernels.hip, argument checks.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <new>

#include "lbml.h"
#include "lbml_launch.hpp"

namespace lbmp {
lb_status abi_fail(lb_status st, const std::string& msg);
lb_status abi_hip_fail(hipError_t e, const char* what);
}  // namespace lbmp

namespace {

using lbmp::abi_fail;
using lbmp::abi_hip_fail;

constexpr size_t kAlign = 256;
constexpr int kLayers = 4;
constexpr int kIn[kLayers] = {lbml::kIn, lbml::kHidden, lbml::kHidden, lbml::kHidden};
constexpr int kInPadded[kLayers] = {lbml::kInPad, lbml::kHidden, lbml::kHidden, lbml::kHidden};
constexpr int kOutN[kLayers] = {lbml::kHidden, lbml::kHidden, lbml::kHidden, lbml::kOut};

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// offsets of W_i and b_i in the flat parameter vector
constexpr size_t w_off(int i)
{
    size_t o = 0;
    for (int j = 0; j < i; ++j) o += (size_t)kOutN[j] * kIn[j] + kOutN[j];
    return o;
}
constexpr size_t b_off(int i) { return w_off(i) + (size_t)kOutN[i] * kIn[i]; }
static_assert(w_off(kLayers) == LBML_PARAMS, "parameter count");

struct Layout {
    size_t theta, m, v, grad, norm, loss, wb[kLayers], x16, z[kLayers], h[kLayers - 1], c, dz[2];
    size_t xg, bg, tg, sched;  // a graph-replayed training step: gathered rows and the device schedule
    size_t total;
};

Layout layout_of(int B)
{
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align_up(bytes);
        return at;
    };
    const size_t P = LBML_PARAMS * sizeof(float);
    L.theta = take(P);
    L.m = take(P);
    L.v = take(P);
    L.grad = take(P);
    L.norm = take(2 * lbml::kIn * sizeof(float));
    L.loss = take(sizeof(float));
    for (int i = 0; i < kLayers; ++i) L.wb[i] = take((size_t)kOutN[i] * kInPadded[i] * 2);
    L.x16 = take((size_t)B * lbml::kInPad * 2);
    for (int i = 0; i < kLayers; ++i) L.z[i] = take((size_t)B * kOutN[i] * 4);
    for (int i = 0; i < kLayers - 1; ++i) L.h[i] = take((size_t)B * lbml::kHidden * 2);
    // GEMM scratch: [B][256] activations or gradients, or the padded [256][32] first-layer weight gradient
    L.c = take((size_t)B * lbml::kHidden * 4);
    L.dz[0] = take((size_t)B * lbml::kHidden * 2);
    L.dz[1] = take((size_t)B * lbml::kHidden * 2);
    L.xg = take((size_t)B * lbml::kIn * 4);
    L.bg = take((size_t)B * lbml::kOut * 4);
    L.tg = take((size_t)B * lbml::kOut * 4);
    L.sched = take(sizeof(lbml::TrainSched));
    L.total = o;
    return L;
}

bool batch_ok(int32_t B) { return B >= 32 && B % 32 == 0 && B <= (1 << 20); }

constexpr double kBeta1 = 0.9, kBeta2 = 0.999;
constexpr float kEps = 1e-8f;

}  // namespace

struct lbml_net {
    int max_batch = 0;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    Layout L{};
    long long t = 0;          // Adam steps taken
    double p1 = 1.0, p2 = 1.0;  // b1^t and b2^t, one FP64 product per step (the device schedule repeats them)
    bool have_grad = false;
    lbml::TrainSched sched_init{};  // host copy of the schedule uploaded before a graph-replayed loop

    float* f(size_t off) { return reinterpret_cast<float*>(ws + off); }
    __bf16* h16(size_t off) { return reinterpret_cast<__bf16*>(ws + off); }
};

namespace {

hipError_t refresh_bf16(lbml_net* n)
{
    hipError_t e = hipSuccess;
    for (int i = 0; i < kLayers && e == hipSuccess; ++i)
        e = lbml::launch_to_bf16(n->f(n->L.theta) + w_off(i), n->h16(n->L.wb[i]), kOutN[i], kIn[i], kInPadded[i],
                                 n->stream);
    return e;
}

// Forward pass; the output layer writes y = network(x) + base (FP32 [B][128]).
hipError_t forward(lbml_net* n, const float* x, const float* base, int B, float* y)
{
    hipError_t e = lbml::launch_pack_input(x, n->f(n->L.norm), n->f(n->L.norm) + lbml::kIn, n->h16(n->L.x16), B,
                                           n->stream);
    const __bf16* hin = n->h16(n->L.x16);
    for (int i = 0; i < kLayers && e == hipSuccess; ++i) {
        const int K = kInPadded[i], N = kOutN[i];
        e = lbml::gemm(hin, K, 1, n->h16(n->L.wb[i]), 1, K, n->f(n->L.c), N, B, N, K, n->stream);
        if (e != hipSuccess) break;
        const bool last = i == kLayers - 1;
        float* z = last ? y : n->f(n->L.z[i]);
        __bf16* hout = last ? nullptr : n->h16(n->L.h[i]);
        e = lbml::launch_bias_act(n->f(n->L.c), n->f(n->L.theta) + b_off(i), last ? base : nullptr, z, hout, B, N,
                                  n->stream);
        hin = hout;
    }
    return e;
}

hipError_t backward(lbml_net* n, const float* target, int B, float* loss)
{
    float* grad = n->f(n->L.grad);
    const float* y = n->f(n->L.z[kLayers - 1]);
    int cur = 0;
    hipError_t e = lbml::launch_mse_grad(y, target, n->h16(n->L.dz[cur]), loss, B, lbml::kOut, n->stream);
    for (int i = kLayers - 1; i >= 0 && e == hipSuccess; --i) {
        const int Kp = kInPadded[i], N = kOutN[i];
        const __bf16* dz = n->h16(n->L.dz[cur]);
        const __bf16* hin = i > 0 ? n->h16(n->L.h[i - 1]) : n->h16(n->L.x16);
        // dW_i[N][Kp] = dZ^T H_in
        float* dw = i > 0 ? grad + w_off(i) : n->f(n->L.c);
        e = lbml::gemm(dz, 1, N, hin, Kp, 1, dw, Kp, N, Kp, B, n->stream);
        if (e == hipSuccess && i == 0) e = lbml::launch_copy_cols(dw, Kp, grad + w_off(0), N, kIn[0], n->stream);
        if (e == hipSuccess) e = lbml::launch_bias_grad(dz, grad + b_off(i), B, N, n->stream);
        if (e != hipSuccess || i == 0) break;
        // dH_{i-1}[B][Kp] = dZ W_i, then dZ_{i-1} = bf16(dH * GELU'(Z_{i-1}))
        e = lbml::gemm(dz, N, 1, n->h16(n->L.wb[i]), Kp, 1, n->f(n->L.c), Kp, B, Kp, N, n->stream);
        if (e == hipSuccess)
            e = lbml::launch_gelu_back(n->f(n->L.c), n->f(n->L.z[i - 1]), n->h16(n->L.dz[cur ^ 1]), B * Kp,
                                       n->stream);
        cur ^= 1;
    }
    return e;
}

lb_status check_net(lbml_net* n, int32_t B, bool train)
{
    if (!n) return abi_fail(LB_EINVAL, "net is NULL");
    if (B <= 0 || B > n->max_batch || B % (train ? 32 : 16))
        return abi_fail(LB_EINVAL, std::string("batch must be a positive multiple of ") + (train ? "32" : "16") +
                                       " not above max_batch");
    return LB_OK;
}

}  // namespace

extern "C" {

size_t lbml_workspace_bytes(int32_t max_batch)
{
    if (!batch_ok(max_batch)) return 0;
    return layout_of(max_batch).total;
}

lb_status lbml_init(lbml_net** out, int32_t max_batch, void* workspace, size_t workspace_bytes,
                    const float* theta0, const double* mu, const double* sd, void* stream)
{
    if (!out) return abi_fail(LB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!batch_ok(max_batch)) return abi_fail(LB_EINVAL, "max_batch must be a positive multiple of 32, <= 2^20");
    if (!workspace || !theta0 || !mu || !sd) return abi_fail(LB_EINVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return abi_fail(LB_EINVAL, "workspace must be 256-byte aligned");
    if (workspace_bytes < lbml_workspace_bytes(max_batch))
        return abi_fail(LB_ENOMEM, "workspace smaller than lbml_workspace_bytes");
    float norm[2 * lbml::kIn];
    for (int k = 0; k < lbml::kIn; ++k) {
        if (!std::isfinite(mu[k]) || !std::isfinite(sd[k]) || !(sd[k] > 0.0))
            return abi_fail(LB_EINVAL, "feature mean must be finite and standard deviation positive");
        norm[k] = (float)mu[k];
        norm[lbml::kIn + k] = (float)(1.0 / sd[k]);
    }
    lbml_net* n = new (std::nothrow) lbml_net{};
    if (!n) return abi_fail(LB_ENOMEM, "host allocation failed");
    n->max_batch = max_batch;
    n->stream = static_cast<hipStream_t>(stream);
    n->ws = static_cast<char*>(workspace);
    n->L = layout_of(max_batch);
    const size_t P = LBML_PARAMS * sizeof(float);
    hipError_t e = hipMemcpyAsync(n->f(n->L.theta), theta0, P, hipMemcpyDeviceToDevice, n->stream);
    if (e == hipSuccess) e = lbml::launch_fill(n->ws + n->L.m, P, n->stream);
    if (e == hipSuccess) e = lbml::launch_fill(n->ws + n->L.v, P, n->stream);
    if (e == hipSuccess) e = lbml::launch_fill(n->ws + n->L.grad, P, n->stream);
    if (e == hipSuccess) e = lbml::launch_fill(n->ws + n->L.wb[0], (size_t)lbml::kHidden * lbml::kInPad * 2, n->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(n->f(n->L.norm), norm, sizeof(norm), hipMemcpyHostToDevice, n->stream);
    if (e == hipSuccess) e = refresh_bf16(n);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    if (e != hipSuccess) {
        delete n;
        return abi_hip_fail(e, "lbml_init");
    }
    *out = n;
    return LB_OK;
}

lb_status lbml_set_params(lbml_net* n, const float* theta)
{
    if (!n || !theta) return abi_fail(LB_EINVAL, "NULL argument");
    hipError_t e = hipMemcpyAsync(n->f(n->L.theta), theta, LBML_PARAMS * sizeof(float), hipMemcpyDeviceToDevice,
                                  n->stream);
    if (e == hipSuccess) e = refresh_bf16(n);
    return e == hipSuccess ? LB_OK : abi_hip_fail(e, "lbml_set_params");
}

lb_status lbml_get_params(lbml_net* n, float* theta)
{
    if (!n || !theta) return abi_fail(LB_EINVAL, "NULL argument");
    hipError_t e = hipMemcpyAsync(theta, n->f(n->L.theta), LBML_PARAMS * sizeof(float), hipMemcpyDeviceToDevice,
                                  n->stream);
    return e == hipSuccess ? LB_OK : abi_hip_fail(e, "lbml_get_params");
}

lb_status lbml_forward(lbml_net* n, const float* x, const float* base, int32_t B, float* y)
{
    lb_status st = check_net(n, B, false);
    if (st != LB_OK) return st;
    if (!x || !y) return abi_fail(LB_EINVAL, "NULL argument");
    hipError_t e = forward(n, x, base, B, y);
    return e == hipSuccess ? LB_OK : abi_hip_fail(e, "lbml_forward");
}

lb_status lbml_loss_grad(lbml_net* n, const float* x, const float* base, const float* target, int32_t B, float* loss,
                         float* grad)
{
    lb_status st = check_net(n, B, true);
    if (st != LB_OK) return st;
    if (!x || !target) return abi_fail(LB_EINVAL, "NULL argument");
    hipError_t e = forward(n, x, base, B, n->f(n->L.z[kLayers - 1]));
    if (e == hipSuccess) e = backward(n, target, B, loss ? loss : n->f(n->L.loss));
    if (e == hipSuccess && grad)
        e = hipMemcpyAsync(grad, n->f(n->L.grad), LBML_PARAMS * sizeof(float), hipMemcpyDeviceToDevice, n->stream);
    if (e != hipSuccess) return abi_hip_fail(e, "lbml_loss_grad");
    n->have_grad = true;
    return LB_OK;
}

lb_status lbml_adam(lbml_net* n, float lr)
{
    if (!n) return abi_fail(LB_EINVAL, "net is NULL");
    if (!n->have_grad) return abi_fail(LB_ESTATE, "no gradient: call lbml_loss_grad first");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return abi_fail(LB_EINVAL, "learning rate must be positive");
    const double p1 = n->p1 * kBeta1, p2 = n->p2 * kBeta2;
    const float c1 = (float)(1.0 - p1), c2 = (float)(1.0 - p2);
    hipError_t e = lbml::launch_adam(n->f(n->L.theta), n->f(n->L.m), n->f(n->L.v), n->f(n->L.grad), LBML_PARAMS, lr,
                                     (float)kBeta1, (float)kBeta2, kEps, c1, c2, n->stream);
    if (e == hipSuccess) e = refresh_bf16(n);
    if (e != hipSuccess) return abi_hip_fail(e, "lbml_adam");
    n->t += 1;
    n->p1 = p1;
    n->p2 = p2;
    return LB_OK;
}

lb_status lbml_train_step(lbml_net* n, const float* x, const float* base, const float* target, int32_t B, float lr,
                          float* loss)
{
    lb_status st = lbml_loss_grad(n, x, base, target, B, loss, nullptr);
    return st == LB_OK ? lbml_adam(n, lr) : st;
}

lb_status lbml_train_steps(lbml_net* n, const float* x_all, const float* base_all, const float* target_all,
                           int32_t rows, const int32_t* idx, const float* lr, int32_t steps, int32_t B, float* loss)
{
    lb_status st = check_net(n, B, true);
    if (st != LB_OK) return st;
    if (steps < 0) return abi_fail(LB_EINVAL, "need steps >= 0");
    if (steps == 0) return LB_OK;
    if (!x_all || !target_all || !idx || !lr) return abi_fail(LB_EINVAL, "NULL argument");
    if (rows < 1) return abi_fail(LB_EINVAL, "need rows >= 1");
    if (!n->stream) return abi_fail(LB_EINVAL, "lbml_train_steps needs the net on a non-null stream (graph capture)");
    hipStream_t s = n->stream;
    auto* sc = reinterpret_cast<lbml::TrainSched*>(n->ws + n->L.sched);
    // the schedule starts at step 0 with the net's Adam state; indices are checked first
    n->sched_init = lbml::TrainSched{};
    n->sched_init.p1 = n->p1;
    n->sched_init.p2 = n->p2;
    hipError_t e = hipMemcpyAsync(sc, &n->sched_init, sizeof(lbml::TrainSched), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = lbml::launch_check_rows(idx, (long long)steps * B, rows, &sc->bad_rows, s);
    int bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, &sc->bad_rows, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return abi_hip_fail(e, "lbml_train_steps");
    if (bad) return abi_fail(LB_EINVAL, "lbml_train_steps: a row index lies outside [0, rows)");

    // one step, captured: schedule, gather, forward, backward, loss record, Adam, bf16 refresh
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return abi_hip_fail(e, "lbml_train_steps (begin capture)");
    float* xg = n->f(n->L.xg);
    float* bg = base_all ? n->f(n->L.bg) : nullptr;
    float* tg = n->f(n->L.tg);
    e = lbml::launch_sched_advance(sc, lr, kBeta1, kBeta2, s);
    if (e == hipSuccess) e = lbml::launch_gather_rows(x_all, base_all, target_all, idx, sc, B, xg, bg, tg, s);
    if (e == hipSuccess) e = forward(n, xg, bg, B, n->f(n->L.z[kLayers - 1]));
    if (e == hipSuccess) e = backward(n, tg, B, n->f(n->L.loss));
    if (e == hipSuccess && loss) e = lbml::launch_record_loss(n->f(n->L.loss), sc, loss, s);
    if (e == hipSuccess)
        e = lbml::launch_adam_sched(n->f(n->L.theta), n->f(n->L.m), n->f(n->L.v), n->f(n->L.grad), LBML_PARAMS, sc,
                                    (float)kBeta1, (float)kBeta2, kEps, s);
    if (e == hipSuccess) e = refresh_bf16(n);
    const hipError_t ec = hipStreamEndCapture(s, &graph);
    if (e == hipSuccess) e = ec;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    for (int32_t i = 0; i < steps && e == hipSuccess; ++i) e = hipGraphLaunch(exec, s);
    const hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess) e = es;
    if (exec) {
        const hipError_t ed = hipGraphExecDestroy(exec);
        if (e == hipSuccess) e = ed;
    }
    if (graph) {
        const hipError_t ed = hipGraphDestroy(graph);
        if (e == hipSuccess) e = ed;
    }
    if (e != hipSuccess) return abi_hip_fail(e, "lbml_train_steps");
    for (int32_t i = 0; i < steps; ++i) {
        n->p1 *= kBeta1;
        n->p2 *= kBeta2;
    }
    n->t += steps;
    n->have_grad = true;
    return LB_OK;
}

lb_status lbml_destroy(lbml_net* n)
{
    delete n;
    return LB_OK;
}

size_t lbml_profile_scratch_bytes(int32_t ny)
{
    if (ny < 2 || ny > (1 << 20)) return 0;
    return (size_t)3 * ny * lbml::kOut * sizeof(double);
}

lb_status lbml_profile_extract(const float* rho, int32_t nx, int32_t ny, double cx, double cy, double R,
                               void* scratch, size_t scratch_bytes, float* logrho, void* stream)
{
    if (!rho || !logrho || !scratch) return abi_fail(LB_EINVAL, "NULL argument");
    if (nx < 2 || ny < 2 || nx > (1 << 20) || ny > (1 << 20) || (long long)nx * ny > (1LL << 31))
        return abi_fail(LB_EINVAL, "bad lattice size");
    if (!std::isfinite(cx) || !std::isfinite(cy) || !std::isfinite(R) || R < 0.0 || R > 1e6)
        return abi_fail(LB_EINVAL, "centre and radius must be finite, 0 <= R <= 1e6");
    if (reinterpret_cast<uintptr_t>(scratch) % 8) return abi_fail(LB_EINVAL, "scratch must be 8-byte aligned");
    if (scratch_bytes < lbml_profile_scratch_bytes(ny))
        return abi_fail(LB_ENOMEM, "scratch smaller than lbml_profile_scratch_bytes(ny)");
    hipError_t e = lbml::launch_profile_extract(rho, nx, ny, cx, cy, R, static_cast<double*>(scratch), logrho,
                                                static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LB_OK : abi_hip_fail(e, "lbml_profile_extract");
}

lb_status lbml_profile_extract_noalloc(const float* rho, int32_t nx, int32_t ny, double cx, double cy, double R,
                                       float* logrho, void* stream)
{
    if (!rho || !logrho) return abi_fail(LB_EINVAL, "NULL argument");
    if (nx < 2 || ny < 2 || nx > (1 << 20) || (long long)nx * ny > (1LL << 31))
        return abi_fail(LB_EINVAL, "bad lattice size");
    if (ny > lbml::static_profile_rows())
        return abi_fail(LB_EINVAL, "ny exceeds the 2048 rows of the static profile scratch (use lbml_profile_extract)");
    if (!std::isfinite(cx) || !std::isfinite(cy) || !std::isfinite(R) || R < 0.0 || R > 1e6)
        return abi_fail(LB_EINVAL, "centre and radius must be finite, 0 <= R <= 1e6");
    hipError_t e = lbml::launch_profile_extract_static(rho, nx, ny, cx, cy, R, logrho, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LB_OK : abi_hip_fail(e, "lbml_profile_extract_noalloc");
}

lb_status lbml_profile_to_rho0(const float* logrho, double R, double cx, double cy, int32_t nx, int32_t ny,
                               float* rho0, void* stream)
{
    if (!rho0 || !logrho) return abi_fail(LB_EINVAL, "NULL argument");
    if (nx < 1 || ny < 1 || ny > 65535 || (long long)nx * ny > (1LL << 31))
        return abi_fail(LB_EINVAL, "bad lattice size");
    if (!std::isfinite(cx) || !std::isfinite(cy) || !std::isfinite(R) || R < 0.0 || R > 1e6)
        return abi_fail(LB_EINVAL, "centre and radius must be finite, 0 <= R <= 1e6");
    hipError_t e = lbml::launch_profile_to_rho0(logrho, R, cx, cy, nx, ny, rho0, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LB_OK : abi_hip_fail(e, "lbml_profile_to_rho0");
}

lb_status lbml_profile_to_rho0_mass(const float* logrho, double R, double cx, double cy, int32_t nx, int32_t ny,
                                    double mass, double* shift, float* rho0, void* stream)
{
    if (!rho0 || !logrho || !shift) return abi_fail(LB_EINVAL, "NULL argument");
    if (nx < 1 || ny < 1 || ny > 65535 || (long long)nx * ny > (1LL << 31))
        return abi_fail(LB_EINVAL, "bad lattice size");
    if (!std::isfinite(cx) || !std::isfinite(cy) || !std::isfinite(R) || R < 0.0 || R > 1e6)
        return abi_fail(LB_EINVAL, "centre and radius must be finite, 0 <= R <= 1e6");
    if (!std::isfinite(mass) || !(mass > 0.0)) return abi_fail(LB_EINVAL, "mass must be positive and finite");
    if (reinterpret_cast<uintptr_t>(shift) % 8) return abi_fail(LB_EINVAL, "shift must be 8-byte aligned");
    hipError_t e = lbml::launch_profile_to_rho0_mass(logrho, R, cx, cy, nx, ny, mass, shift, rho0,
                                                     static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LB_OK : abi_hip_fail(e, "lbml_profile_to_rho0_mass");
}

lb_status lbml_profile_levels(const float* L, const float* x, int32_t B, double* levels, void* stream)
{
    if (!L || !x || !levels) return abi_fail(LB_EINVAL, "NULL argument");
    if (B < 1 || B > (1 << 20)) return abi_fail(LB_EINVAL, "need 1 <= B <= 2^20 profiles");
    if (reinterpret_cast<uintptr_t>(levels) % 8) return abi_fail(LB_EINVAL, "levels must be 8-byte aligned");
    hipError_t e = lbml::launch_profile_levels(L, x, B, levels, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LB_OK : abi_hip_fail(e, "lbml_profile_levels");
}

lb_status lbml_profile_anchor(float* L, const float* x, const double* target, int32_t B, void* stream)
{
    if (!L || !x || !target) return abi_fail(LB_EINVAL, "NULL argument");
    if (B < 1 || B > (1 << 20)) return abi_fail(LB_EINVAL, "need 1 <= B <= 2^20 profiles");
    if (reinterpret_cast<uintptr_t>(target) % 8) return abi_fail(LB_EINVAL, "target must be 8-byte aligned");
    hipError_t e = lbml::launch_profile_anchor(L, x, target, B, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LB_OK : abi_hip_fail(e, "lbml_profile_anchor");
}

lb_status lbml_gemm_bf16(const void* A, int64_t sam, int64_t sak, const void* B, int64_t sbk, int64_t sbn, float* C,
                         int32_t ldc, int32_t M, int32_t N, int32_t K, void* stream)
{
    if (!A || !B || !C) return abi_fail(LB_EINVAL, "NULL argument");
    if (M <= 0 || N <= 0 || K <= 0 || M % 16 || N % 16 || K % 32)
        return abi_fail(LB_EINVAL, "M, N must be positive multiples of 16 and K of 32");
    if (ldc < N) return abi_fail(LB_EINVAL, "ldc < N");
    hipError_t e = lbml::gemm(static_cast<const __bf16*>(A), sam, sak, static_cast<const __bf16*>(B), sbk, sbn, C,
                              ldc, M, N, K, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LB_OK : abi_hip_fail(e, "lbml_gemm_bf16");
}

}  // extern "C"
