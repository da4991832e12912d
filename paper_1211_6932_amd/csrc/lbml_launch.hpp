// Host-side launchers of the learned-initialiser kernels (lbml_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace lbml {

constexpr int kIn = 4;       // inputs: a, T/T_c, R, nu_g/nu_l (standardised)
constexpr int kInPad = 32;   // first-layer depth padded to one matrix-core step
constexpr int kHidden = 256;
constexpr int kOut = 128;    // log-density samples across the interface
constexpr double kSmooth = 1e-4;  // weight of the profile fit's smoothness term

// Device state of a training loop replayed from a graph: the step being run
// (cur), the next one, the running powers b1^t and b2^t of Adam's bias
// correction (FP64, multiplied once per step as the host does), and the current
// step's learning rate and FP32 bias corrections.
struct TrainSched {
    int cur, next;
    double p1, p2;
    float lr, c1, c2;
    int bad_rows;
};

hipError_t gemm(const __bf16* A, long long sam, long long sak, const __bf16* B, long long sbk, long long sbn,
                float* C, int ldc, int M, int N, int K, hipStream_t s);
hipError_t launch_pack_input(const float* x, const float* mu, const float* inv_sd, __bf16* x16, int B,
                             hipStream_t s);
hipError_t launch_bias_act(const float* C, const float* b, const float* base, float* Z, __bf16* H, int B, int N,
                           hipStream_t s);
hipError_t launch_mse_grad(const float* Y, const float* T, __bf16* dY, float* loss, int B, int N, hipStream_t s);
hipError_t launch_gelu_back(const float* dH, const float* Z, __bf16* dZ, int n, hipStream_t s);
hipError_t launch_bias_grad(const __bf16* dZ, float* db, int B, int N, hipStream_t s);
hipError_t launch_copy_cols(const float* src, int lds, float* dst, int rows, int cols, hipStream_t s);
hipError_t launch_adam(float* p, float* m, float* v, const float* g, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2, hipStream_t s);
hipError_t launch_adam_sched(float* p, float* m, float* v, const float* g, int n, const TrainSched* sc, float b1,
                             float b2, float eps, hipStream_t s);
hipError_t launch_sched_advance(TrainSched* sc, const float* lr, double b1, double b2, hipStream_t s);
hipError_t launch_gather_rows(const float* x_all, const float* base_all, const float* t_all, const int* idx,
                              const TrainSched* sc, int B, float* x, float* base, float* t, hipStream_t s);
hipError_t launch_record_loss(const float* loss, const TrainSched* sc, float* loss_out, hipStream_t s);
hipError_t launch_check_rows(const int* idx, long long n, int rows, int* flag, hipStream_t s);
hipError_t launch_to_bf16(const float* src, __bf16* dst, int rows, int cols, int ldd, hipStream_t s);
hipError_t launch_fill(void* p, size_t bytes, hipStream_t s);
hipError_t launch_profile_extract(const float* rho, int nx, int ny, double cx, double cy, double R, double* part,
                                  float* logrho, hipStream_t s);
// The same fit with its row partials in the library's static device scratch (ny up to
// static_profile_rows()); hipErrorInvalidValue for a larger ny.
hipError_t launch_profile_extract_static(const float* rho, int nx, int ny, double cx, double cy, double R,
                                         float* logrho, hipStream_t s);
int static_profile_rows();
hipError_t launch_profile_to_rho0(const float* logrho, double R, double cx, double cy, int nx, int ny, float* rho0,
                                  hipStream_t s);
hipError_t launch_profile_to_rho0_mass(const float* logrho, double R, double cx, double cy, int nx, int ny,
                                       double mass, double* shift, float* rho0, hipStream_t s);
hipError_t launch_profile_levels(const float* L, const float* x, int B, double* lev, hipStream_t s);
hipError_t launch_profile_anchor(float* L, const float* x, const double* target, int B, hipStream_t s);

}  // namespace lbml
