// lbml_kernels.hip -- gfx950 kernels of the learned droplet initialiser: a
// 4 -> 256 -> 256 -> 256 -> 128 MLP with bf16 matrix-core products (FP32
// accumulation, FP32 master weights, Adam), plus the two profile kernels that
// connect it to the lattice (radial log-density samples <-> density field).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "lbml_launch.hpp"

namespace lbml {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// C[M][N] (FP32, row stride ldc) = sum_k A(m, k) B(k, n) with A(m, k) at
// A[m * sam + k * sak] and B(k, n) at B[k * sbk + n * sbn] (bf16).  One
// wavefront per 16 x 16 tile of C, K consumed 32 at a time by
// v_mfma_f32_16x16x32_bf16: lane l holds row (or column) l % 16 and the eight
// consecutive k values 8 (l / 16) .. 8 (l / 16) + 7 of each operand; the
// accumulator holds rows 4 (l / 16) .. 4 (l / 16) + 3 of column l % 16.
// AV / BV: the operand is contiguous in k (sak == 1 / sbk == 1) with 16-byte
// aligned rows, so a lane's eight k values are one 16-byte load; otherwise eight
// 2-byte loads.  Either way the matrix cores see the same values.
// M, N multiples of 16 and K a multiple of 32 (checked by the launcher).
template <bool AV, bool BV>
__global__ __launch_bounds__(256) void gemm_bf16(const __bf16* __restrict__ A, long long sam,
                                                 long long sak, const __bf16* __restrict__ B,
                                                 long long sbk, long long sbn, float* __restrict__ C,
                                                 int ldc, int M, int N, int K)
{
    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tiles_n = N / 16;
    if (tile >= (M / 16) * tiles_n) return;
    const int m0 = (tile / tiles_n) * 16, n0 = (tile % tiles_n) * 16;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    const __bf16* arow = A + (long long)(m0 + r) * sam;
    const __bf16* bcol = B + (long long)(n0 + r) * sbn;
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 a, b;
        if constexpr (AV) {
            a = *reinterpret_cast<const bf16x8*>(arow + k0 + kq);
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) a[i] = arow[(long long)(k0 + kq + i) * sak];
        }
        if constexpr (BV) {
            b = *reinterpret_cast<const bf16x8*>(bcol + k0 + kq);
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) b[i] = bcol[(long long)(k0 + kq + i) * sbk];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) C[(long long)(m0 + (lane >> 4) * 4 + i) * ldc + n0 + r] = acc[i];
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_prime(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// x [B][4] raw features -> bf16 [B][32]: standardised (x - mu) / sd, then
// zero-padded to the matrix-core depth.
__global__ void pack_input(const float* __restrict__ x, const float* __restrict__ mu,
                           const float* __restrict__ inv_sd, __bf16* __restrict__ x16, int B)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * kInPad) return;
    const int m = i / kInPad, k = i % kInPad;
    x16[i] = static_cast<__bf16>(k < kIn ? (x[m * kIn + k] - mu[k]) * inv_sd[k] : 0.0f);
}

__global__ void fill_zero(unsigned int* __restrict__ p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Z = C + b; H = bf16(GELU(Z)) (hidden layers), or Y = C + b + base (output
// layer: H == nullptr; base [B][N] may be nullptr).
__global__ void bias_act(const float* __restrict__ C, const float* __restrict__ bias,
                         const float* __restrict__ base, float* __restrict__ Z, __bf16* __restrict__ H, int B, int N)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * N) return;
    float z = C[i] + bias[i % N];
    if (base) z += base[i];
    Z[i] = z;
    if (H) H[i] = static_cast<__bf16>(gelu(z));
}

// dY = bf16(2 (Y - T) / (B N)); loss = mean (Y - T)^2, one workgroup, fixed order.
__global__ __launch_bounds__(1024) void mse_grad(const float* __restrict__ Y, const float* __restrict__ T,
                                                 __bf16* __restrict__ dY, float* __restrict__ loss, int B, int N)
{
    __shared__ float part[1024];
    const float scale = 2.0f / (float)(B * N);
    float acc = 0.0f;
    for (int i = threadIdx.x; i < B * N; i += 1024) {
        const float d = Y[i] - T[i];
        dY[i] = static_cast<__bf16>(scale * d);
        acc += d * d;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) loss[0] = part[0] / (float)(B * N);
}

// dZ = bf16(dH * GELU'(Z)).
__global__ void gelu_back(const float* __restrict__ dH, const float* __restrict__ Z, __bf16* __restrict__ dZ,
                          int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dZ[i] = static_cast<__bf16>(dH[i] * gelu_prime(Z[i]));
}

// db[n] = sum_m dZ[m][n] (sequential in m: deterministic).
__global__ void bias_grad(const __bf16* __restrict__ dZ, float* __restrict__ db, int B, int N)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float acc = 0.0f;
    int m = 0;
    // 16 rows loaded ahead, then added in row order: the loads overlap, the sum and
    // its rounding stay those of the plain sequential loop
    for (; m + 16 <= B; m += 16) {
        float v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = static_cast<float>(dZ[(long long)(m + j) * N + n]);
#pragma unroll
        for (int j = 0; j < 16; ++j) acc += v[j];
    }
    for (; m < B; ++m) acc += static_cast<float>(dZ[(long long)m * N + n]);
    db[n] = acc;
}

// dst[n][k] = src[n][k] for k < cols (drops the zero padding of the first layer).
__global__ void copy_cols(const float* __restrict__ src, int lds, float* __restrict__ dst, int rows, int cols)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < rows * cols) dst[i] = src[(i / cols) * lds + i % cols];
}

// Adam on the FP32 master parameters (the bf16 copies of the weights are
// refreshed by to_bf16 afterwards).  c1, c2: the bias corrections 1 - b1^t, 1 - b2^t.
__device__ __forceinline__ void adam_update(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                            const float* __restrict__ g, int i, float lr, float b1, float b2,
                                            float eps, float c1, float c2)
{
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                     const float* __restrict__ g, int n, float lr, float b1, float b2, float eps, float c1,
                     float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) adam_update(p, m, v, g, i, lr, b1, b2, eps, c1, c2);
}

// The same update with the learning rate and bias corrections of the current
// step read from the device schedule (training loops replayed from a graph).
__global__ void adam_sched(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ g, int n, const TrainSched* __restrict__ sc, float b1,
                           float b2, float eps)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) adam_update(p, m, v, g, i, sc->lr, b1, b2, eps, sc->c1, sc->c2);
}

// One thread: advance the schedule to the next step: step index, learning rate
// lr[step], running powers b1^t, b2^t (FP64 products, as the host keeps them) and
// the bias corrections rounded to FP32.
__global__ void sched_advance(TrainSched* __restrict__ sc, const float* __restrict__ lr, double b1, double b2)
{
    const int s = sc->next;
    sc->cur = s;
    sc->next = s + 1;
    sc->p1 *= b1;
    sc->p2 *= b2;
    sc->lr = lr[s];
    sc->c1 = (float)(1.0 - sc->p1);
    sc->c2 = (float)(1.0 - sc->p2);
}

// Rows idx[cur][i] of the training set into the step's buffers: features [B][4],
// base [B][128] (if base_all is not NULL) and target [B][128].  One workgroup of
// 128 threads per row.
__global__ __launch_bounds__(kOut) void gather_rows(const float* __restrict__ x_all, const float* __restrict__ base_all,
                                                    const float* __restrict__ t_all, const int* __restrict__ idx,
                                                    const TrainSched* __restrict__ sc, int B, float* __restrict__ x,
                                                    float* __restrict__ base, float* __restrict__ t)
{
    const int i = blockIdx.x, k = threadIdx.x;
    const long long row = idx[(long long)sc->cur * B + i];
    if (k < kIn) x[i * kIn + k] = x_all[row * kIn + k];
    if (base_all) base[i * kOut + k] = base_all[row * kOut + k];
    t[i * kOut + k] = t_all[row * kOut + k];
}

// loss_out[cur] = loss (one thread).
__global__ void record_loss(const float* __restrict__ loss, const TrainSched* __restrict__ sc,
                            float* __restrict__ loss_out)
{
    loss_out[sc->cur] = loss[0];
}

// flag[0] = 1 if some idx[j], j < n, lies outside [0, rows).
__global__ void check_rows(const int* __restrict__ idx, long long n, int rows, int* __restrict__ flag)
{
    for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (long long)gridDim.x * blockDim.x)
        if (idx[j] < 0 || idx[j] >= rows) flag[0] = 1;
}

__global__ void to_bf16(const float* __restrict__ src, __bf16* __restrict__ dst, int rows, int cols, int ldd)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < rows * cols) dst[(i / cols) * ldd + i % cols] = static_cast<__bf16>(src[i]);
}

// ---------------------------------------------------------------- profiles
// Sample radii r_k = R + (k - 63.5) / 2, k = 0..127 (a 64-cell window centred
// on the interface).  A profile L (log densities at r_k) defines the field
// log rho0(d) = (1 - t) L_j + t L_{j+1} with s = (d - r_0) / 0.5 clamped to
// [0, 127], j = min(floor(s), 126), t = s - j, d the minimum-image distance.

__device__ __forceinline__ double min_image(double d, int n)
{
    d = fabs(d);
    return fmin(d, n - d);
}

// Hat coordinates (j, t) of distance d.
__device__ __forceinline__ void hat_of(double d, double r0, int& j, double& t)
{
    double s = (d - r0) * 2.0;
    s = fmin(fmax(s, 0.0), (double)(kOut - 1));
    j = min((int)s, kOut - 2);
    t = s - j;
}

// Least-squares fit, stage 1: row y's contributions to the normal equations
// (H^T H) L = H^T log rho.  Thread k accumulates, in x order, the diagonal
// (k, k), the upper off-diagonal (k, k+1) and the right-hand side of sample k
// over the sites of the row.  part: [3][ny][128] doubles.
__global__ __launch_bounds__(kOut) void profile_rows(const float* __restrict__ rho, int nx, int ny, double cx,
                                                     double cy, double r0, double* __restrict__ part)
{
    const int k = threadIdx.x;
    const int y = blockIdx.x;
    const double dy = min_image(y - cy, ny);
    const float* row = rho + (long long)y * nx;
    double a = 0.0, e = 0.0, b = 0.0;
    for (int x = 0; x < nx; ++x) {
        const double dx = min_image(x - cx, nx);
        int j;
        double t;
        hat_of(sqrt(dx * dx + dy * dy), r0, j, t);
        if (j == k) {
            const double v = log((double)row[x]);
            a += (1.0 - t) * (1.0 - t);
            e += (1.0 - t) * t;
            b += (1.0 - t) * v;
        } else if (j + 1 == k) {
            const double v = log((double)row[x]);
            a += t * t;
            b += t * v;
        }
    }
    const long long plane = (long long)ny * kOut;
    part[(long long)y * kOut + k] = a;
    part[plane + (long long)y * kOut + k] = e;
    part[2 * plane + (long long)y * kOut + k] = b;
}

// Stage 2 (one workgroup): sum the rows in order, add lam * (graph Laplacian
// of the sample path), solve the symmetric positive-definite tridiagonal
// system (Thomas algorithm, FP64) and write L as FP32.
__global__ __launch_bounds__(kOut) void profile_solve(const double* __restrict__ part, int ny,
                                                      float* __restrict__ logrho)
{
    __shared__ double A[kOut], E[kOut], Bv[kOut], Cp[kOut], Dp[kOut];
    const int k = threadIdx.x;
    const long long plane = (long long)ny * kOut;
    double a = 0.0, e = 0.0, b = 0.0;
    for (int y = 0; y < ny; ++y) {
        a += part[(long long)y * kOut + k];
        e += part[plane + (long long)y * kOut + k];
        b += part[2 * plane + (long long)y * kOut + k];
    }
    if (k > 0) a += kSmooth;
    if (k < kOut - 1) {
        a += kSmooth;
        e -= kSmooth;
    }
    A[k] = a;
    E[k] = e;  // coupling of samples k and k + 1 (unused for k = 127)
    Bv[k] = b;
    __syncthreads();
    if (k == 0) {
        Cp[0] = E[0] / A[0];
        Dp[0] = Bv[0] / A[0];
        for (int i = 1; i < kOut; ++i) {
            const double m = A[i] - E[i - 1] * Cp[i - 1];
            Cp[i] = i < kOut - 1 ? E[i] / m : 0.0;
            Dp[i] = (Bv[i] - E[i - 1] * Dp[i - 1]) / m;
        }
        for (int i = kOut - 2; i >= 0; --i) Dp[i] -= Cp[i] * Dp[i + 1];
    }
    __syncthreads();
    logrho[k] = (float)Dp[k];
}

// rho0(x, y) = exp((1 - t) L_j + t L_{j+1}) at the minimum-image distance of
// (x, y) from (cx, cy); the sample radii are moved outwards by shift[0] when
// shift is not NULL.
__global__ void profile_to_rho0(const float* __restrict__ logrho, double r0, const double* __restrict__ shift,
                                double cx, double cy, int nx, int ny, float* __restrict__ rho0)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= nx) return;
    const double dx = min_image(x - cx, nx), dy = min_image(y - cy, ny);
    int j;
    double t;
    hat_of(sqrt(dx * dx + dy * dy), r0 + (shift ? shift[0] : 0.0), j, t);
    rho0[(long long)y * nx + x] = (float)exp((1.0 - t) * logrho[j] + t * logrho[j + 1]);
}

constexpr int kMassThreads = 1024;
constexpr int kMassIters = 60;
constexpr double kMaxShift = 8.0;

// Bisection for the outward shift delta in [-8, 8] at which the profile's field
// has total mass `mass` (the mass grows with delta for a profile that falls
// outwards).  One workgroup; FP64 site sums reduced in a fixed tree order.
// out[0] = delta, out[1] = the field's mass at delta.
__global__ __launch_bounds__(kMassThreads) void profile_mass_shift(const float* __restrict__ logrho, double r0,
                                                                   double cx, double cy, int nx, int ny,
                                                                   double mass, double* __restrict__ out)
{
    __shared__ float L[kOut];
    __shared__ double part[kMassThreads];
    __shared__ double lohi[2];
    const int tid = threadIdx.x;
    if (tid < kOut) L[tid] = logrho[tid];
    if (tid == 0) {
        lohi[0] = -kMaxShift;
        lohi[1] = kMaxShift;
    }
    __syncthreads();
    const long long n = (long long)nx * ny;
    double m = 0.0;
    for (int it = 0; it <= kMassIters; ++it) {
        const double delta = 0.5 * (lohi[0] + lohi[1]);
        double acc = 0.0;
        for (long long i = tid; i < n; i += kMassThreads) {
            const int x = (int)(i % nx), y = (int)(i / nx);
            const double dx = min_image(x - cx, nx), dy = min_image(y - cy, ny);
            int j;
            double t;
            hat_of(sqrt(dx * dx + dy * dy), r0 + delta, j, t);
            acc += exp((1.0 - t) * (double)L[j] + t * (double)L[j + 1]);
        }
        part[tid] = acc;
        __syncthreads();
        for (int s = kMassThreads / 2; s > 0; s >>= 1) {
            if (tid < s) part[tid] += part[tid + s];
            __syncthreads();
        }
        m = part[0];
        if (tid == 0 && it < kMassIters) {
            if (m < mass) lohi[0] = delta;
            else lohi[1] = delta;
        }
        __syncthreads();
        if (it == kMassIters && tid == 0) {
            out[0] = delta;
            out[1] = m;
        }
    }
}

// ---------------------------------------------------------------- liquid level
// Bands of a profile around radius R (d_k = (k - 63.5) / 2): inner = samples with
// d_k <= -min(12, R / 2), outer = samples with d_k >= 12.  Inside a relaxed droplet
// the density is the Laplace-shifted liquid density (Sec. IV.A-B); the inner band
// holds it, the outer band the vapour.

constexpr double kBand = 12.0;

// Means of the sample's log density over the two bands, for the workgroup of kOut
// threads that holds one profile (thread k = sample k).  FP64 tree sums in a fixed
// order.  An empty band gives NaN (0 / 0).
__device__ void band_means(double v, double R, double& m_in, double& m_out)
{
    __shared__ double part[4][kOut];
    const int k = threadIdx.x;
    const double d = (k - 63.5) * 0.5;
    const bool in = d <= -fmin(kBand, 0.5 * R);
    const bool out = d >= kBand;
    part[0][k] = in ? v : 0.0;
    part[1][k] = in ? 1.0 : 0.0;
    part[2][k] = out ? v : 0.0;
    part[3][k] = out ? 1.0 : 0.0;
    __syncthreads();
    for (int s = kOut / 2; s > 0; s >>= 1) {
        if (k < s) {
#pragma unroll
            for (int q = 0; q < 4; ++q) part[q][k] += part[q][k + s];
        }
        __syncthreads();
    }
    m_in = part[0][0] / part[1][0];
    m_out = part[2][0] / part[3][0];
    __syncthreads();  // part is reused by the next call
}

// lev[b] = (inner, outer) band means of profile b; R = x[b][2].
__global__ __launch_bounds__(kOut) void profile_levels(const float* __restrict__ L, const float* __restrict__ x,
                                                       double* __restrict__ lev)
{
    const long long b = blockIdx.x;
    const int k = threadIdx.x;
    double m_in, m_out;
    band_means((double)L[b * kOut + k], (double)x[b * kIn + 2], m_in, m_out);
    if (k == 0) {
        lev[2 * b] = m_in;
        lev[2 * b + 1] = m_out;
    }
}

// Profile b pinned to the inner level target[b], in place: with rho = exp(L),
// rho_in / rho_out = exp of the band means and rho* = exp(target),
// rho'_k = rho_out + (rho_k - rho_out) g, g = (rho* - rho_out) / (rho_in - rho_out),
// then rho'_k = rho* on the inner band.  The profile is left as it is when the
// target or g is not finite or some rho'_k <= 0.
__global__ __launch_bounds__(kOut) void profile_anchor(float* __restrict__ L, const float* __restrict__ x,
                                                       const double* __restrict__ target)
{
    const long long b = blockIdx.x;
    const int k = threadIdx.x;
    const double R = (double)x[b * kIn + 2];
    const double v = (double)L[b * kOut + k];
    double m_in, m_out;
    band_means(v, R, m_in, m_out);
    const double lev = target[b];
    const double r_in = exp(m_in), r_out = exp(m_out), r_t = exp(lev);
    const double g = (r_t - r_out) / (r_in - r_out);
    const bool in = (k - 63.5) * 0.5 <= -fmin(kBand, 0.5 * R);
    const double rho = in ? r_t : r_out + (exp(v) - r_out) * g;
    const bool usable = isfinite(lev) && isfinite(g);
    const int bad = __syncthreads_or(!(rho > 0.0));
    if (usable && !bad) L[b * kOut + k] = (float)log(rho);
}

// ---------------------------------------------------------------- launchers

static unsigned grid1(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_profile_levels(const float* L, const float* x, int B, double* lev, hipStream_t s)
{
    hipLaunchKernelGGL(profile_levels, dim3(B), dim3(kOut), 0, s, L, x, lev);
    return hipGetLastError();
}

hipError_t launch_profile_anchor(float* L, const float* x, const double* target, int B, hipStream_t s)
{
    hipLaunchKernelGGL(profile_anchor, dim3(B), dim3(kOut), 0, s, L, x, target);
    return hipGetLastError();
}

// An operand that is contiguous in k with 16-byte aligned rows loads eight k values at once.
static bool rows_of_8(const __bf16* P, long long s_row, long long s_k)
{
    return s_k == 1 && s_row % 8 == 0 && reinterpret_cast<uintptr_t>(P) % 16 == 0;
}

hipError_t gemm(const __bf16* A, long long sam, long long sak, const __bf16* B, long long sbk, long long sbn,
                float* C, int ldc, int M, int N, int K, hipStream_t s)
{
    if (M % 16 || N % 16 || K % 32 || M <= 0 || N <= 0 || K <= 0) return hipErrorInvalidValue;
    const long long tiles = (long long)(M / 16) * (N / 16);
    const bool av = rows_of_8(A, sam, sak), bv = rows_of_8(B, sbn, sbk);
    auto kern = av ? (bv ? gemm_bf16<true, true> : gemm_bf16<true, false>)
                   : (bv ? gemm_bf16<false, true> : gemm_bf16<false, false>);
    hipLaunchKernelGGL(kern, dim3(grid1(tiles, 4)), dim3(256), 0, s, A, sam, sak, B, sbk, sbn, C, ldc, M, N, K);
    return hipGetLastError();
}

hipError_t launch_pack_input(const float* x, const float* mu, const float* inv_sd, __bf16* x16, int B,
                             hipStream_t s)
{
    hipLaunchKernelGGL(pack_input, dim3(grid1((long long)B * kInPad, 256)), dim3(256), 0, s, x, mu, inv_sd, x16, B);
    return hipGetLastError();
}

// bytes must be a multiple of 4
hipError_t launch_fill(void* p, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_zero, dim3(grid1((long long)n, 256)), dim3(256), 0, s, static_cast<unsigned int*>(p), n);
    return hipGetLastError();
}

hipError_t launch_bias_act(const float* C, const float* b, const float* base, float* Z, __bf16* H, int B, int N,
                           hipStream_t s)
{
    hipLaunchKernelGGL(bias_act, dim3(grid1((long long)B * N, 256)), dim3(256), 0, s, C, b, base, Z, H, B, N);
    return hipGetLastError();
}

hipError_t launch_mse_grad(const float* Y, const float* T, __bf16* dY, float* loss, int B, int N, hipStream_t s)
{
    hipLaunchKernelGGL(mse_grad, dim3(1), dim3(1024), 0, s, Y, T, dY, loss, B, N);
    return hipGetLastError();
}

hipError_t launch_gelu_back(const float* dH, const float* Z, __bf16* dZ, int n, hipStream_t s)
{
    hipLaunchKernelGGL(gelu_back, dim3(grid1(n, 256)), dim3(256), 0, s, dH, Z, dZ, n);
    return hipGetLastError();
}

hipError_t launch_bias_grad(const __bf16* dZ, float* db, int B, int N, hipStream_t s)
{
    hipLaunchKernelGGL(bias_grad, dim3(grid1(N, 256)), dim3(256), 0, s, dZ, db, B, N);
    return hipGetLastError();
}

hipError_t launch_copy_cols(const float* src, int lds, float* dst, int rows, int cols, hipStream_t s)
{
    hipLaunchKernelGGL(copy_cols, dim3(grid1((long long)rows * cols, 256)), dim3(256), 0, s, src, lds, dst, rows, cols);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, float* m, float* v, const float* g, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2, hipStream_t s)
{
    hipLaunchKernelGGL(adam, dim3(grid1(n, 256)), dim3(256), 0, s, p, m, v, g, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_adam_sched(float* p, float* m, float* v, const float* g, int n, const TrainSched* sc, float b1,
                             float b2, float eps, hipStream_t s)
{
    hipLaunchKernelGGL(adam_sched, dim3(grid1(n, 256)), dim3(256), 0, s, p, m, v, g, n, sc, b1, b2, eps);
    return hipGetLastError();
}

hipError_t launch_sched_advance(TrainSched* sc, const float* lr, double b1, double b2, hipStream_t s)
{
    hipLaunchKernelGGL(sched_advance, dim3(1), dim3(1), 0, s, sc, lr, b1, b2);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const float* x_all, const float* base_all, const float* t_all, const int* idx,
                              const TrainSched* sc, int B, float* x, float* base, float* t, hipStream_t s)
{
    hipLaunchKernelGGL(gather_rows, dim3(B), dim3(kOut), 0, s, x_all, base_all, t_all, idx, sc, B, x, base, t);
    return hipGetLastError();
}

hipError_t launch_record_loss(const float* loss, const TrainSched* sc, float* loss_out, hipStream_t s)
{
    hipLaunchKernelGGL(record_loss, dim3(1), dim3(1), 0, s, loss, sc, loss_out);
    return hipGetLastError();
}

hipError_t launch_check_rows(const int* idx, long long n, int rows, int* flag, hipStream_t s)
{
    hipLaunchKernelGGL(check_rows, dim3(256), dim3(256), 0, s, idx, n, rows, flag);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float* src, __bf16* dst, int rows, int cols, int ldd, hipStream_t s)
{
    hipLaunchKernelGGL(to_bf16, dim3(grid1((long long)rows * cols, 256)), dim3(256), 0, s, src, dst, rows, cols, ldd);
    return hipGetLastError();
}

hipError_t launch_profile_extract(const float* rho, int nx, int ny, double cx, double cy, double R, double* part,
                                  float* logrho, hipStream_t s)
{
    const double r0 = R - 0.25 * (kOut - 1);
    hipLaunchKernelGGL(profile_rows, dim3(ny), dim3(kOut), 0, s, rho, nx, ny, cx, cy, r0, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(profile_solve, dim3(1), dim3(kOut), 0, s, part, ny, logrho);
    return hipGetLastError();
}

// Scratch of the allocation-free profile fit: the [3][ny][128] FP64 row partials for
// ny <= kStaticProfileRows.  Each GPU the library runs on holds its own copy until the
// process ends.  In host code the name `scratch` is only a stand-in for the symbol:
// its device address comes from hipGetSymbolAddress, once per device.
constexpr int kStaticProfileRows = 2048;  // the limit lbml.h states for lbml_profile_extract_noalloc
static __device__ __align__(256) double scratch[3 * kStaticProfileRows * kOut];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on the current device, looked up with that device
// current on the first call and kept per device.
hipError_t static_profile_scratch(double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

int static_profile_rows() { return kStaticProfileRows; }

hipError_t launch_profile_extract_static(const float* rho, int nx, int ny, double cx, double cy, double R,
                                         float* logrho, hipStream_t s)
{
    if (ny > kStaticProfileRows) return hipErrorInvalidValue;
    double* part = nullptr;
    const hipError_t e = static_profile_scratch(&part);
    if (e != hipSuccess) return e;
    // profile_rows writes every partial that profile_solve reads: nothing to clear
    return launch_profile_extract(rho, nx, ny, cx, cy, R, part, logrho, s);
}

hipError_t launch_profile_to_rho0(const float* logrho, double R, double cx, double cy, int nx, int ny, float* rho0,
                                  hipStream_t s)
{
    const double r0 = R - 0.25 * (kOut - 1);
    hipLaunchKernelGGL(profile_to_rho0, dim3(grid1(nx, 256), ny), dim3(256), 0, s, logrho, r0,
                       static_cast<const double*>(nullptr), cx, cy, nx, ny, rho0);
    return hipGetLastError();
}

hipError_t launch_profile_to_rho0_mass(const float* logrho, double R, double cx, double cy, int nx, int ny,
                                       double mass, double* shift, float* rho0, hipStream_t s)
{
    const double r0 = R - 0.25 * (kOut - 1);
    hipLaunchKernelGGL(profile_mass_shift, dim3(1), dim3(kMassThreads), 0, s, logrho, r0, cx, cy, nx, ny, mass, shift);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(profile_to_rho0, dim3(grid1(nx, 256), ny), dim3(256), 0, s, logrho, r0,
                       static_cast<const double*>(shift), cx, cy, nx, ny, rho0);
    return hipGetLastError();
}

}  // namespace lbml
