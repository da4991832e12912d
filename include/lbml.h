/*
 * lbml.h -- C ABI of the learned droplet initialiser in liblbmp.so.
 *
 * The paper initialises a droplet with the tanh profile of Eq. (31) between
 * the Maxwell coexistence densities (Sec. IV.A) and lets the lattice relax to
 * its own equilibrium: interface shape, bulk densities shifted by the
 * droplet's Laplace pressure (Sec. IV.B) and the residual spurious currents
 * (Sec. IV.B, Table I).  This part replaces
 * the tanh profile by the relaxed profile predicted by a small network trained
 * on profiles that the lattice itself produced, so that a run starts close to
 * its equilibrium.  The tanh profile stays the fallback; the lattice run
 * measures the prediction's error.
 *
 * Network: 4 features (a, T/T_c, R, nu_g/nu_l), standardised with a mean and
 * standard deviation fixed at lbml_init -> 3 hidden layers of 256 units with
 * the exact GELU, x/2 (1 + erf(x / sqrt 2)) -> 128 linear outputs
 * y_k = log rho(r_k), r_k = R + (k - 63.5) / 2, k = 0..127 (radial samples
 * across the interface, 64 lattice units wide).  Matrix products take bf16
 * operands (weights, layer inputs, output and pre-activation gradients) and
 * accumulate in FP32 on the matrix cores; master weights, biases, activations
 * before rounding, gradients and Adam moments are FP32.  Loss: mean squared
 * error over batch and outputs.
 *
 * Parameter vector (FP32, 165,760 values, in this order):
 *   W1[256][4] b1[256] W2[256][256] b2[256] W3[256][256] b3[256] W4[128][256] b4[128]
 *
 * Conventions: as in lbmp.h (lb_status results, lb_last_error(), caller-owned
 * device buffers, asynchronous on the net's stream unless stated).
 */
#ifndef LBML_H
#define LBML_H

#include "lbmp.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { LBML_IN = 4, LBML_HIDDEN = 256, LBML_OUT = 128, LBML_PARAMS = 165760 };

typedef struct lbml_net lbml_net; /* opaque host-side handle */

/* Device workspace for batches of up to max_batch samples (pure host; 0 if
 * max_batch is not a positive multiple of 32 or exceeds 2^20). */
size_t lbml_workspace_bytes(int32_t max_batch);

/* Create a network in `workspace` (device, 256-byte aligned, at least
 * lbml_workspace_bytes(max_batch) bytes, owned by the caller and used until
 * lbml_destroy).  theta0: device [LBML_PARAMS] FP32 initial parameters.
 * mu, sd: host [4] feature means and standard deviations (sd > 0).
 * Adam moments and step counter start at zero.  Synchronises the stream. */
lb_status lbml_init(lbml_net** out, int32_t max_batch, void* workspace, size_t workspace_bytes,
                    const float* theta0, const double* mu, const double* sd, void* stream);

/* theta: device [LBML_PARAMS] FP32.  set also refreshes the bf16 weights and
 * keeps the Adam state. */
lb_status lbml_set_params(lbml_net* net, const float* theta);
lb_status lbml_get_params(lbml_net* net, float* theta);

/* y (device [B][128] FP32) = network(x) + base, x device [B][4] raw
 * features, base device [B][128] or NULL (zero): the network can learn a
 * correction to a known profile, such as the tanh start of Eq. (31).
 * B: multiple of 16, at most max_batch. */
lb_status lbml_forward(lbml_net* net, const float* x, const float* base, int32_t B, float* y);

/* Forward and backward over one batch: loss (device, 1 float; may be NULL) =
 * mean squared error of network(x) + base against target (device [B][128]);
 * the gradient is kept in the net and copied to grad (device [LBML_PARAMS])
 * if grad != NULL.  B: multiple of 32, at most max_batch. */
lb_status lbml_loss_grad(lbml_net* net, const float* x, const float* base, const float* target, int32_t B,
                         float* loss, float* grad);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the
 * gradient of the last lbml_loss_grad, then refresh the bf16 weights. */
lb_status lbml_adam(lbml_net* net, float lr);

/* lbml_loss_grad followed by lbml_adam. */
lb_status lbml_train_step(lbml_net* net, const float* x, const float* base, const float* target, int32_t B,
                          float lr, float* loss);

/* A training loop on the device: `steps` Adam steps, step s on the minibatch of
 * the B rows idx[s][0..B-1] (device [steps][B] int32, each in [0, rows)) of
 * x_all (device [rows][4] raw features), base_all (device [rows][128], or NULL
 * for zero) and target_all (device [rows][128]), at learning rate lr[s] (device
 * [steps] FP32).  loss (device [steps] FP32, or NULL) receives each step's loss.
 * The kernels of one step (row gather, forward, backward, Adam, bf16 refresh)
 * are captured once into a HIP graph and replayed `steps` times; the step index,
 * learning rate and Adam's bias correction come from a schedule kept on the
 * device.  The result is bitwise that of `steps` calls of lbml_train_step on the
 * gathered rows.  B: multiple of 32, at most max_batch.  The net's stream must
 * not be the null stream (it is captured).  The indices are checked first
 * (LB_EINVAL, nothing trained, if one is out of range).  steps = 0 returns LB_OK
 * at once (the array arguments may then be NULL).  Synchronises the stream. */
lb_status lbml_train_steps(lbml_net* net, const float* x_all, const float* base_all, const float* target_all,
                           int32_t rows, const int32_t* idx, const float* lr, int32_t steps, int32_t B, float* loss);

/* Release the handle (not the caller's workspace). */
lb_status lbml_destroy(lbml_net* net);

/* Profiles.  A profile L (device [128] FP32) defines the density field
 * rho(x, y) = exp((1 - t) L_j + t L_{j+1}), where d is the minimum-image
 * distance of (x, y) from the centre (cx, cy), s = (d - r_0) / 0.5 clamped to
 * [0, 127], j = min(floor(s), 126), t = s - j: linear interpolation in d,
 * end values held inside r_0 and beyond r_127.
 *
 * lbml_profile_extract: the profile whose field best fits the density field
 * rho (device [ny][nx] FP32, periodic) in least squares of log density over
 * all sites, plus 1e-4 sum_k (L_{k+1} - L_k)^2 (a weak smoothness term that
 * only matters where no site falls, r_k < 0).  FP64 normal equations, summed
 * in a fixed order (bitwise reproducible), solved by tridiagonal elimination.
 * scratch: device, 8-byte aligned, at least lbml_profile_scratch_bytes(ny).
 * Asynchronous on `stream`. */
size_t lbml_profile_scratch_bytes(int32_t ny);
lb_status lbml_profile_extract(const float* rho, int32_t nx, int32_t ny, double cx, double cy, double R,
                               void* scratch, size_t scratch_bytes, float* logrho, void* stream);

/* lbml_profile_extract without a scratch argument, for callers that cannot allocate
 * device memory (code under graph capture, serving loops, harnesses that forbid
 * hipMalloc).  The row partials live in a static device array of the library,
 * 3 x 2048 x 128 doubles (6 MiB, held by each GPU the library runs on until the process
 * ends); ny > 2048 returns LB_EINVAL.  The call allocates nothing: its first call on a
 * device looks up that device's copy of the array once.  Results are bitwise those of
 * lbml_profile_extract.  Every call on one GPU shares the array: calls that overlap on
 * one GPU (different streams or host threads) race and must be serialised by the caller.
 * Asynchronous on `stream`. */
lb_status lbml_profile_extract_noalloc(const float* rho, int32_t nx, int32_t ny, double cx, double cy, double R,
                                       float* logrho, void* stream);

/* lbml_profile_to_rho0: the field of a profile, into rho0 (device [ny][nx]
 * FP32).  Asynchronous on `stream`. */
lb_status lbml_profile_to_rho0(const float* logrho, double R, double cx, double cy, int32_t nx, int32_t ny,
                               float* rho0, void* stream);

/* lbml_profile_to_rho0_mass: the field of the profile moved outwards by the
 * distance delta (|delta| <= 8, bisection, FP64 site sums in a fixed order) at
 * which its total mass sum rho0 equals `mass`, for instance the mass of the
 * tanh start of the same droplet, so that both starts relax to the same
 * equilibrium.  shift: device, 2 doubles, receives (delta, achieved mass);
 * delta is clamped to [-8, 8] if the mass is not reachable.  One workgroup
 * does the search: cost ~60 passes over the lattice.  Asynchronous. */
lb_status lbml_profile_to_rho0_mass(const float* logrho, double R, double cx, double cy, int32_t nx, int32_t ny,
                                    double mass, double* shift, float* rho0, void* stream);

/* Liquid level.  Inside a relaxed droplet the density is uniform, the coexisting
 * liquid density (Sec. IV.A) shifted by the droplet's Laplace pressure
 * (Sec. IV.B); the start's error in that density sets how far its pressure jump
 * starts from the relaxed one.  The network's samples carry independent errors of
 * about 1e-3 in log density, so the interior level is predicted by a separate FP64
 * linear model and the network's profile is pinned to it.
 *
 * Bands of a profile around radius R (sample offsets d_k = (k - 63.5) / 2):
 * inner = samples with d_k <= -min(12, R / 2), never empty for 0 <= R <= 63.5;
 * outer = samples with d_k >= 12 (k = 88..127).
 *
 * lbml_profile_levels: levels (device [B][2] FP64, 8-byte aligned) = the means of
 * L_k (device [B][128] FP32) over the inner and over the outer band of each
 * profile, R = x[b][2] (device [B][4] FP32 raw features); FP64 sums in a fixed
 * order; NaN for an empty band.  1 <= B <= 2^20.  Asynchronous on `stream`. */
lb_status lbml_profile_levels(const float* L, const float* x, int32_t B, double* levels, void* stream);

/* lbml_profile_anchor: profile b of L (device [B][128] FP32, in place) pinned to
 * the inner level target[b] (device [B] FP64, 8-byte aligned): with
 * rho_k = exp(L_k), rho_in / rho_out = exp of the band means and
 * rho* = exp(target[b]), rho'_k = rho_out + (rho_k - rho_out) g with
 * g = (rho* - rho_out) / (rho_in - rho_out), then rho'_k = rho* on the inner
 * band; L_k = log rho'_k in FP32 (the arithmetic is FP64).  The map is affine in
 * density: the interface shape and the vapour end are kept and the inner band
 * becomes exactly flat.  A profile whose target or g is not finite, or whose
 * rho'_k would not all be positive, is left as it is.  R = x[b][2].
 * 1 <= B <= 2^20.  Asynchronous on `stream`. */
lb_status lbml_profile_anchor(float* L, const float* x, const double* target, int32_t B, void* stream);

/* Level model: y(x) = sum_c coef[c] T_i(z_a) T_j(z_t) T_k(z_u) T_l(z_v) over the
 * Chebyshev polynomials T_n, i <= 2, j <= 6, k <= 3, l <= 1, column
 * c = ((i * 7 + j) * 4 + k) * 2 + l, of the features (a, T/T_c, u = 1/R,
 * nu_g/nu_l); z = 2 (v - lo) / (hi - lo) - 1 clamped to [-1, 1] (z = 0 when
 * hi == lo), lo and hi being in the variable u for R. */
enum { LBML_LEVEL_TERMS = 168 };
typedef struct lbml_level_model {
    double lo[LBML_IN];
    double hi[LBML_IN];
    double coef[LBML_LEVEL_TERMS];
} lbml_level_model;

/* Host, FP64.  Fit: lo and hi = the range of each feature over the rows of x
 * (host [n][4], finite, R > 0), coef = the least-squares solution of
 * [A; sqrt(lam) I] c = [y; 0] with A the [n][168] basis matrix and
 * lam = 1e-12 trace(A^T A) / 168 (a ridge term that keeps a feature with a single
 * value, or n < 168 rows, solvable), by Householder QR.  y: host [n].
 * 1 <= n <= 262144.  LB_EINVAL for bad arguments, LB_ENOMEM if the host working
 * matrix ((n + 168) x 168 doubles) cannot be allocated. */
lb_status lbml_level_fit(const double* x, const double* y, int32_t n, lbml_level_model* model);

/* Host, FP64: y[i] (host [n]) = the model at row i of x (host [n][4], finite,
 * R > 0).  0 <= n <= 2^30. */
lb_status lbml_level_eval(const lbml_level_model* model, const double* x, int32_t n, double* y);

/* Building block, exported for tests: C[M][N] (device FP32, row stride ldc) =
 * sum_k A(m, k) B(k, n) with bf16 device operands A(m, k) = A[m sam + k sak]
 * and B(k, n) = B[k sbk + n sbn].  M, N multiples of 16, K a multiple of 32. */
lb_status lbml_gemm_bf16(const void* A, int64_t sam, int64_t sak, const void* B, int64_t sbk, int64_t sbn,
                         float* C, int32_t ldc, int32_t M, int32_t N, int32_t K, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LBML_H */
