// lbmp_abi.cpp -- host runtime behind the C ABI of include/lbmp.h.
//
// Responsibilities: parameter validation (pure host), FP64 derivation of the
// FP32 kernel constants, carving of the caller-owned workspace, graph capture
// and replay of step loops, error state.  Every numerical step of the method
// runs in the kernels of d2q9_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbmp.h"
#include "d2q9_launch.hpp"

namespace {

thread_local std::string g_last_error;

lb_status fail(lb_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

lb_status hip_fail(hipError_t e, const char* what)
{
    return fail(LB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
constexpr int kDiagStripRows = 32;
constexpr int kMinStripRows = 3;
constexpr int kBatchPersistentRows = 24;  // measured best (one workgroup walks a whole lattice)
constexpr int kDefaultBand = 1;
constexpr int kDefaultGraphChunk = 32;
constexpr int kMaxSide = 1 << 20;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_bytes(int store) { return store == LB_STORE_F32 ? 4 : 2; }

bool local_density(int store) { return store == LB_STORE_F16_LOCAL || store == LB_STORE_BF16_LOCAL; }

// storage-type row slots per lattice row: nine population rows, plus an FP32
// density row (two 16-bit slots) for the local-density encodings, or a bf16
// density-scale row (one slot) for the destination-scaled encoding
int row_slots(int store)
{
    if (local_density(store)) return 11;
    return store == LB_STORE_F16_DEST ? 10 : 9;
}

// bytes per site of the exported density plane (0: none)
size_t density_plane_bytes(int store)
{
    if (local_density(store)) return sizeof(float);
    return store == LB_STORE_F16_DEST ? 2 : 0;
}

// Elements per population row.  The rows are packed without padding: the nine (ten,
// eleven) population rows of a lattice row, and consecutive lattice rows, then form one
// contiguous stream.  Measured on the 512-lattice sweep (sides 64-512): FP32 73.3k
// MLUPS with rows packed against 63.4k with rows padded to 64 elements, whose holes
// break the stream (destination-scaled FP16: 96.9k against 88.9k).  The local-density
// encodings round to an even count so that their FP32 density row stays 4-byte aligned.
int pitch_of(int nx, int store) { return local_density(store) ? (nx + 1) / 2 * 2 : nx; }

// Output columns per wavefront strip of the one-column kernels for this stencil.
int tile_width(const lb_params& p) { return p.stencil == LB_STENCIL_MULTIRANGE ? lbmp::kMrTileW : lbmp::kTileW; }

struct Layout {
    size_t flag_off, dout_off, partial_off, f_off[2], total, buf_bytes;
    int diag_tiles;
};

Layout layout_of(const lb_params& p)
{
    Layout L{};
    const int pitch = pitch_of(p.nx, p.store);
    L.buf_bytes = align_up((size_t)row_slots(p.store) * p.ny * pitch * elem_bytes(p.store), kAlign);
    const int tw = tile_width(p);
    const int tx = (p.nx + tw - 1) / tw;
    const int ty = (p.ny + kDiagStripRows - 1) / kDiagStripRows;
    L.diag_tiles = tx * ty;
    L.flag_off = 0;
    L.dout_off = kAlign;
    L.partial_off = 2 * kAlign;
    size_t off = align_up(L.partial_off + (size_t)L.diag_tiles * lbmp::kDiagFields * sizeof(double), kAlign);
    L.f_off[0] = off;
    L.f_off[1] = off + L.buf_bytes;
    L.total = off + 2 * L.buf_bytes;
    return L;
}

bool finite_all(std::initializer_list<double> v)
{
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

bool rate_ok(double s) { return s > 0.0 && s < 2.0; }

lb_status validate(const lb_params* p)
{
    if (!p) return fail(LB_EINVAL, "params is NULL");
    if (p->nx < 3 || p->ny < 3 || p->nx > kMaxSide || p->ny > kMaxSide)
        return fail(LB_EINVAL, "nx and ny must lie in [3, 2^20]");
    if ((long long)p->nx * p->ny > (1LL << 31)) return fail(LB_EINVAL, "nx * ny exceeds 2^31 sites");
    if ((long long)pitch_of(p->nx, p->store) * row_slots(p->store) * (p->store == LB_STORE_F32 ? 4 : 2) >= (1LL << 32))
        return fail(LB_EINVAL, "a lattice row must stay below 4 GiB");
    if (p->bc != LB_BC_PERIODIC && p->bc != LB_BC_WALLS_Y) return fail(LB_EINVAL, "unknown bc");
    if (p->stencil != LB_STENCIL_NEAREST && p->stencil != LB_STENCIL_MULTIRANGE)
        return fail(LB_EINVAL, "unknown stencil");
    if (p->stencil == LB_STENCIL_MULTIRANGE && p->store != LB_STORE_F32)
        return fail(LB_EINVAL, "the 24-site stencil runs with LB_STORE_F32 only");
    if (p->store < LB_STORE_F32 || p->store > LB_STORE_F16_DEST) return fail(LB_EINVAL, "unknown store");
    if (!finite_all({p->a, p->b, p->R, p->T, p->G, p->sigma, p->s_rho, p->s_e, p->s_zeta, p->s_j,
                     p->s_q, p->nu_l, p->nu_g, p->rho_switch, p->rho_ref, p->psi_eps}))
        return fail(LB_EINVAL, "non-finite parameter");
    if (p->psi_form == LB_PSI_CS) {
        if (!(p->b > 0.0) || !(p->T > 0.0) || !(p->R > 0.0) || !(p->a >= 0.0))
            return fail(LB_EINVAL, "need a >= 0, b > 0, R > 0, T > 0");
    } else if (p->psi_form == LB_PSI_SS) {
        if (!(p->psi_eps >= 0.0)) return fail(LB_EINVAL, "need psi_eps >= 0 (Eq. 23)");
    } else {
        return fail(LB_EINVAL, "unknown psi_form");
    }
    if (!(p->G < 0.0)) return fail(LB_EINVAL, "need G < 0 (Eq. 24 radicand)");
    if (!(p->sigma >= 0.0)) return fail(LB_EINVAL, "need sigma >= 0");
    if (!rate_ok(p->s_rho) || !rate_ok(p->s_e) || !rate_ok(p->s_zeta) || !rate_ok(p->s_j) ||
        !rate_ok(p->s_q))
        return fail(LB_EINVAL, "relaxation rates must lie in (0, 2)");
    if (!(p->nu_l > 0.0) || !(p->nu_g > 0.0)) return fail(LB_EINVAL, "viscosities must be > 0");
    if (!(p->rho_switch >= 0.0)) return fail(LB_EINVAL, "rho_switch must be >= 0");
    if ((p->store == LB_STORE_F16_OFFSET || p->store == LB_STORE_BF16_OFFSET) && !(p->rho_ref >= 0.0))
        return fail(LB_EINVAL, "rho_ref must be >= 0");
    return LB_OK;
}

lbmp::PsiConst psi_const(const lb_params& p)
{
    return lbmp::PsiConst{p.b / 4.0, p.R * p.T, p.a, p.G, p.psi_eps, p.psi_form};
}

lbmp::StepConst derive(const lb_params& p, int strip_rows, int band = 1)
{
    lbmp::StepConst k{};
    k.nx = p.nx;
    k.ny = p.ny;
    k.pitch = pitch_of(p.nx, p.store);
    k.strip_rows = strip_rows;
    k.band = band;
    k.tiles_x = (p.nx + tile_width(p) - 1) / tile_width(p);
    k.tiles_y = (p.ny + strip_rows - 1) / strip_rows;
    k.row_stride = (long long)row_slots(p.store) * k.pitch;
    k.b4 = (float)(p.b / 4.0);
    k.RT = (float)(p.R * p.T);
    k.a = (float)p.a;
    k.two_over_G = (float)(2.0 / p.G);
    k.negG = (float)(-p.G);
    k.rho_switch = (float)p.rho_switch;
    k.a_e = (float)(p.s_e / 36.0);
    k.b_e = (float)(6.0 * (1.0 - 0.5 * p.s_e) / 36.0);
    k.a_z = (float)(p.s_zeta / 36.0);
    k.b_z = (float)(6.0 * (1.0 - 0.5 * p.s_zeta) / 36.0);
    k.a_q = (float)(p.s_q / 12.0);
    k.b_q = (float)((1.0 - 0.5 * p.s_q) / 12.0);
    const double s_nu_l = 1.0 / (3.0 * p.nu_l + 0.5), s_nu_g = 1.0 / (3.0 * p.nu_g + 0.5);
    k.a_nu_l = (float)(s_nu_l / 4.0);
    k.b_nu_l = (float)((1.0 - 0.5 * s_nu_l) / 2.0);
    k.a_nu_g = (float)(s_nu_g / 4.0);
    k.b_nu_g = (float)((1.0 - 0.5 * s_nu_g) / 2.0);
    const double G2 = p.G * p.G;
    k.c_e = (float)(12.0 * p.sigma * G2 * p.s_e / 36.0);
    k.c_z = (float)(12.0 * p.sigma * G2 * p.s_zeta / 36.0);
    k.psi_form = p.psi_form;
    k.stencil = p.stencil;
    k.psi_eps = (float)p.psi_eps;
    k.inv_psi_eps = p.psi_eps > 0.0 ? (float)(1.0 / p.psi_eps) : 0.0f;
    static const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    const bool global16 = p.store == LB_STORE_F16_OFFSET || p.store == LB_STORE_BF16_OFFSET;
    for (int a = 0; a < 9; ++a) k.off[a] = global16 ? (float)(w[a] * p.rho_ref) : 0.0f;
    return k;
}

// Strip height for the step kernel.  Short strips are fastest on large grids
// even though they re-read two halo rows per strip: the tiles are numbered
// row-band by row-band, so the resident wavefronts work on a narrow band of
// rows at any moment (good DRAM-page and last-level-cache locality, halo rows
// shared by neighbouring strips while they are still cached).  Grids too small
// to give every resident wavefront a strip of kMinStripRows rows use shorter
// strips, down to 2 rows.
int auto_strip_rows(const lb_params& p)
{
    // preferred height (measured on the 8192 x 4096 splash): 3 rows for FP32;
    // the issue-bound 16-bit encodings gain from fewer recomputed halo rows:
    // 4 rows for the source-density ones, 8 for the global offsets and the
    // destination-scaled one with one column per lane, 5 for the latter with two
    const bool pair = lbmp::pair_step(p.store, p.nx);
    int preferred = kMinStripRows;
    if (p.stencil == LB_STENCIL_MULTIRANGE)
        preferred = 8;  // two halo rows a side: taller strips pull fewer extra rows
    else if (pair)
        preferred = 5;
    else if (p.store == LB_STORE_F16_DEST || p.store == LB_STORE_F16_OFFSET || p.store == LB_STORE_BF16_OFFSET)
        preferred = 8;
    else if (p.store == LB_STORE_F16_LOCAL || p.store == LB_STORE_BF16_LOCAL)
        preferred = 4;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
        return preferred;
    const bool walls = p.bc == LB_BC_WALLS_Y;
    const int nb = std::max(1, pair ? lbmp::pair_blocks_per_cu(walls) : lbmp::step_blocks_per_cu(p.store, walls));
    const long long resident = (long long)nb * (pair ? lbmp::kPairWaves : lbmp::step_waves_per_block(p.store)) * ncu;
    const int tile_w = pair ? lbmp::kPairTileW : lbmp::kTileW;
    const long long tiles_x = (p.nx + tile_w - 1) / tile_w;
    const long long strips_wanted = (resident + tiles_x - 1) / tiles_x;
    const long long h = std::max<long long>(2, p.ny / strips_wanted);
    return (int)std::min<long long>(h, preferred);
}

}  // namespace

namespace lbmp {
// Error reporting shared with the learned-initialiser entry points (the same
// thread-local message is behind lb_last_error()).
lb_status abi_fail(lb_status st, const std::string& msg) { return fail(st, msg); }
lb_status abi_hip_fail(hipError_t e, const char* what) { return hip_fail(e, what); }
}  // namespace lbmp

struct lb_ctx {
    lb_params p;
    Layout L;
    lbmp::StepConst k;   // step launches
    lbmp::StepConst kd;  // moments / diagnostics launches
    char* ws;
    void* f[2];
    int* flag;
    double* dout;
    double* partial;
    int cur;
    int64_t t;
    hipStream_t stream;
    int graph_chunk;
    hipGraph_t graph[2];
    hipGraphExec_t exec[2];
    bool poisoned;
};

namespace {

void drop_graphs(lb_ctx* c)
{
    for (int i = 0; i < 2; ++i) {
        if (c->exec[i]) (void)hipGraphExecDestroy(c->exec[i]);
        if (c->graph[i]) (void)hipGraphDestroy(c->graph[i]);
        c->exec[i] = nullptr;
        c->graph[i] = nullptr;
    }
}

lb_status step_direct(lb_ctx* c, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        hipError_t e = lbmp::launch_step(c->p.store, c->p.bc == LB_BC_WALLS_Y, c->f[c->cur],
                                         c->f[c->cur ^ 1], c->k, c->flag, c->stream);
        if (e != hipSuccess) {
            c->poisoned = true;
            return hip_fail(e, "step launch");
        }
        c->cur ^= 1;
        c->t += 1;
    }
    return LB_OK;
}

lb_status build_graph(lb_ctx* c, int from)
{
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    int cur = from;
    hipError_t le = hipSuccess;
    for (int i = 0; i < c->graph_chunk && le == hipSuccess; ++i) {
        le = lbmp::launch_step(c->p.store, c->p.bc == LB_BC_WALLS_Y, c->f[cur], c->f[cur ^ 1], c->k,
                               c->flag, c->stream);
        cur ^= 1;
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->stream, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(le, "step launch during capture");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    c->graph[from] = g;
    c->exec[from] = x;
    return LB_OK;
}

lb_status read_flag(lb_ctx* c, int* host_flag)
{
    hipError_t e = hipMemcpyAsync(host_flag, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        c->poisoned = true;
        return hip_fail(e, "reading the device flag");
    }
    return LB_OK;
}

}  // namespace

extern "C" {

lb_status lb_validate_params(const lb_params* p) { return validate(p); }

size_t lb_workspace_bytes(const lb_params* p)
{
    if (validate(p) != LB_OK) return 0;
    return layout_of(*p).total;
}

size_t lb_state_bytes(const lb_params* p)
{
    if (validate(p) != LB_OK) return 0;
    return (size_t)9 * p->nx * p->ny * elem_bytes(p->store) + (size_t)p->nx * p->ny * density_plane_bytes(p->store);
}

}  // extern "C"

namespace {

// Create a context on `workspace` and launch the initial state; with
// sync == false the caller synchronises and checks the flag (batched init).
lb_status init_ctx(lb_ctx** out, const lb_params* p, void* workspace, size_t workspace_bytes,
                   const float* rho0, const float* ux0, const float* uy0, void* stream, bool sync)
{
    if (!out) return fail(LB_EINVAL, "out is NULL");
    *out = nullptr;
    lb_status st = validate(p);
    if (st != LB_OK) return st;
    if (!workspace || !rho0) return fail(LB_EINVAL, "workspace and rho0 must be non-NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(LB_EINVAL, "workspace must be 256-byte aligned");
    Layout L = layout_of(*p);
    if (workspace_bytes < L.total)
        return fail(LB_ENOMEM, "workspace smaller than lb_workspace_bytes");

    lb_ctx* c = new (std::nothrow) lb_ctx{};
    if (!c) return fail(LB_ENOMEM, "host allocation failed");
    c->p = *p;
    c->L = L;
    c->k = derive(*p, auto_strip_rows(*p), kDefaultBand);
    c->kd = derive(*p, kDiagStripRows);
    c->ws = static_cast<char*>(workspace);
    c->flag = reinterpret_cast<int*>(c->ws + L.flag_off);
    c->dout = reinterpret_cast<double*>(c->ws + L.dout_off);
    c->partial = reinterpret_cast<double*>(c->ws + L.partial_off);
    c->f[0] = c->ws + L.f_off[0];
    c->f[1] = c->ws + L.f_off[1];
    c->stream = static_cast<hipStream_t>(stream);
    c->graph_chunk = kDefaultGraphChunk;

    hipError_t e = hipMemsetAsync(c->flag, 0, kAlign, c->stream);
    if (e == hipSuccess)
        e = lbmp::launch_init(p->store, p->bc == LB_BC_WALLS_Y, rho0, ux0, uy0, c->f[0], c->k,
                              lbmp::InitConst{psi_const(*p)}, c->flag, c->stream);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "init launch");
    }
    if (sync) {
        int hf = 0;
        st = read_flag(c, &hf);
        if (st != LB_OK) {
            delete c;
            return st;
        }
        if (hf & lbmp::kFlagBadInput) {
            delete c;
            return fail(LB_EINVAL, "rho0/u0 out of range (need finite, rho > 0, b rho/4 < 1, psi^2 > 0)");
        }
    }
    c->cur = 0;
    c->t = 0;
    *out = c;
    return LB_OK;
}

}  // namespace

extern "C" {

lb_status lb_init(lb_ctx** out, const lb_params* p, void* workspace, size_t workspace_bytes,
                  const float* rho0, const float* ux0, const float* uy0, void* stream)
{
    lb_status st = init_ctx(out, p, workspace, workspace_bytes, rho0, ux0, uy0, stream, true);
    if (st == LB_OK) g_last_error.clear();
    return st;
}

lb_status lb_step(lb_ctx* c, int64_t n)
{
    if (!c) return fail(LB_EINVAL, "ctx is NULL");
    if (c->poisoned) return fail(LB_ESTATE, "context poisoned by an earlier failure");
    if (n < 0) return fail(LB_EINVAL, "nsteps must be >= 0");
    if (c->stream != nullptr) {
        while (n >= c->graph_chunk) {
            if (!c->exec[c->cur]) {
                lb_status st = build_graph(c, c->cur);
                if (st != LB_OK) {
                    c->poisoned = true;
                    return st;
                }
            }
            hipError_t e = hipGraphLaunch(c->exec[c->cur], c->stream);
            if (e != hipSuccess) {
                c->poisoned = true;
                return hip_fail(e, "hipGraphLaunch");
            }
            n -= c->graph_chunk;
            c->t += c->graph_chunk;  // chunk is even: the state returns to buffer cur
        }
    }
    return step_direct(c, n);
}

lb_status lb_moments(lb_ctx* c, float* rho, float* ux, float* uy)
{
    if (!c) return fail(LB_EINVAL, "ctx is NULL");
    if (c->poisoned) return fail(LB_ESTATE, "context poisoned by an earlier failure");
    hipError_t e = lbmp::launch_moments(c->p.store, c->p.bc == LB_BC_WALLS_Y, c->f[c->cur], c->kd,
                                        c->flag, rho, ux, uy, c->stream);
    if (e != hipSuccess) return hip_fail(e, "moments launch");
    return LB_OK;
}

static lbmp::DiagConst diag_const(const lb_ctx* c, const lb_region* in, const lb_region* outr)
{
    return lbmp::DiagConst{in->cx, in->cy, in->r_min, in->r_max,
                           outr->cx, outr->cy, outr->r_min, outr->r_max,
                           psi_const(c->p), c->p.bc == LB_BC_PERIODIC ? 1 : 0};
}

// Host lb_diag from the finalised sums [mass, mom_x, mom_y, sum p_in, sum p_out,
// sum rho_in, sum rho_out, n_in, n_out, max|u|] and the device flag word.
static void fill_diag(const lb_ctx* c, const double* h, int hf, lb_diag* d)
{
    std::memset(d, 0, sizeof(*d));
    d->mass = h[0];
    d->mom_x = h[1];
    d->mom_y = h[2];
    d->n_in = h[7];
    d->n_out = h[8];
    d->p_in = h[7] > 0 ? h[3] / h[7] : NAN;
    d->p_out = h[8] > 0 ? h[4] / h[8] : NAN;
    d->rho_in = h[7] > 0 ? h[5] / h[7] : NAN;
    d->rho_out = h[8] > 0 ? h[6] / h[8] : NAN;
    d->dp = d->p_in - d->p_out;
    d->max_u = h[9];
    d->unstable = hf & lbmp::kFlagUnstable;
    d->step = c->t;
}

lb_status lb_diagnostics(lb_ctx* c, const lb_region* in, const lb_region* outr, lb_diag* d)
{
    if (!c || !in || !outr || !d) return fail(LB_EINVAL, "NULL argument");
    if (c->poisoned) return fail(LB_ESTATE, "context poisoned by an earlier failure");
    hipError_t e = lbmp::launch_diag(c->p.store, c->p.bc == LB_BC_WALLS_Y, c->f[c->cur], c->kd, c->flag,
                                     diag_const(c, in, outr), c->partial, c->dout, c->stream);
    double h[lbmp::kDiagFields];
    int hf = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(h, c->dout, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&hf, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        c->poisoned = true;
        return hip_fail(e, "diagnostics");
    }
    fill_diag(c, h, hf, d);
    if (d->unstable) {
        c->poisoned = true;
        return fail(LB_EUNSTABLE, "unstable site (non-finite rho or psi^2 <= 0) since init");
    }
    return LB_OK;
}

lb_status lb_check(lb_ctx* c)
{
    if (!c) return fail(LB_EINVAL, "ctx is NULL");
    if (c->poisoned) return fail(LB_ESTATE, "context poisoned by an earlier failure");
    int hf = 0;
    lb_status st = read_flag(c, &hf);
    if (st != LB_OK) return st;
    if (hf & lbmp::kFlagUnstable) {
        c->poisoned = true;
        return fail(LB_EUNSTABLE, "unstable site (non-finite rho or psi^2 <= 0) since init");
    }
    return LB_OK;
}

int64_t lb_time(const lb_ctx* c) { return c ? c->t : -1; }

// The exported state is [9][ny][nx] (then [ny][nx] FP32 densities for the
// local-density encodings, or [ny][nx] bf16 scales for the destination-scaled
// one); the stored one is [ny][row_slots][pitch].
static hipError_t copy_state(lb_ctx* c, void* dst, const void* src, bool out)
{
    const size_t eb = elem_bytes(c->p.store);
    const size_t nx = c->p.nx, ny = c->p.ny, pitch = c->k.pitch;
    const size_t row = (size_t)row_slots(c->p.store) * pitch * eb;
    char* buf = static_cast<char*>(out ? const_cast<void*>(src) : dst);
    char* ext = static_cast<char*>(out ? dst : const_cast<void*>(src));
    hipError_t e = hipSuccess;
    for (int a = 0; a < 9 && e == hipSuccess; ++a) {
        char* b = buf + a * pitch * eb;
        char* x = ext + a * ny * nx * eb;
        e = out ? hipMemcpy2DAsync(x, nx * eb, b, row, nx * eb, ny, hipMemcpyDeviceToDevice, c->stream)
                : hipMemcpy2DAsync(b, row, x, nx * eb, nx * eb, ny, hipMemcpyDeviceToDevice, c->stream);
    }
    const size_t db = density_plane_bytes(c->p.store);
    if (e == hipSuccess && db) {
        char* b = buf + 9 * pitch * eb;
        char* x = ext + 9 * ny * nx * eb;
        e = out ? hipMemcpy2DAsync(x, nx * db, b, row, nx * db, ny, hipMemcpyDeviceToDevice, c->stream)
                : hipMemcpy2DAsync(b, row, x, nx * db, nx * db, ny, hipMemcpyDeviceToDevice, c->stream);
    }
    return e;
}

lb_status lb_get_state(lb_ctx* c, void* dst)
{
    if (!c || !dst) return fail(LB_EINVAL, "NULL argument");
    hipError_t e = copy_state(c, dst, c->f[c->cur], true);
    if (e != hipSuccess) return hip_fail(e, "lb_get_state copy");
    return LB_OK;
}

lb_status lb_set_state(lb_ctx* c, const void* src, int64_t t)
{
    if (!c || !src) return fail(LB_EINVAL, "NULL argument");
    if (t < 0) return fail(LB_EINVAL, "t must be >= 0");
    hipError_t e = copy_state(c, c->f[0], src, false);
    if (e != hipSuccess) return hip_fail(e, "lb_set_state copy");
    c->cur = 0;
    c->t = t;
    return LB_OK;
}

lb_status lb_set_launch(lb_ctx* c, int32_t strip_rows, int32_t band, int32_t graph_chunk)
{
    if (!c) return fail(LB_EINVAL, "ctx is NULL");
    if (strip_rows < -1 || band < -1 || graph_chunk < 0) return fail(LB_EINVAL, "invalid launch parameter");
    if (graph_chunk != 0 && (graph_chunk < 2 || graph_chunk % 2))
        return fail(LB_EINVAL, "graph_chunk must be even and >= 2");
    drop_graphs(c);
    int rows = c->k.strip_rows, bd = c->k.band;
    if (strip_rows > 0) rows = strip_rows;
    if (strip_rows == -1) rows = auto_strip_rows(c->p);
    if (band > 0) bd = band;
    if (band == -1) bd = kDefaultBand;
    c->k = derive(c->p, rows, bd);
    if (graph_chunk > 0) c->graph_chunk = graph_chunk;
    return LB_OK;
}

lb_status lb_destroy(lb_ctx* c)
{
    if (!c) return LB_OK;
    drop_graphs(c);
    delete c;
    return LB_OK;
}

const char* lb_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------------ batched lattices

namespace {

// Default strip heights of the stepwise batch, per kernel group, measured on the
// 512-lattice sweep (sides 64-512, packed rows, MI355X), MLUPS by strip rows:
//   FP32, one column per lane:         2: 73.5k  3: 67.6k  5: 59.7k  8: 54.2k
//   destination-scaled FP16 (two columns per lane for even nx, one for odd nx, both
//   groups at the same height):        2: 81.2k  3: 92.1k  5: 98.2k  8: 100.7k
//   source-density FP16:               3: 77.5k  5: 80.1k  8: 79.6k
// A height per lattice-width class, chosen from uniform batches of each width, ran
// slower on the mix (FP32 70.9k): the strips resident at any moment then cover
// different row bands.  lb_batch_tune replaces the defaults by timings on the device
// at hand.
constexpr int kMaxStripRows = 64;
constexpr int kTuneMaxRows = 8;

int default_batch_rows(int store)
{
    if (store == LB_STORE_F16_DEST) return 8;
    if (store == LB_STORE_F16_LOCAL) return 5;
    return 2;
}

}  // namespace

struct lb_batch {
    int n;
    int mode;                        // LB_BATCH_STEPWISE or LB_BATCH_PERSISTENT
    int fixed_rows;                  // > 0: every lattice walks strips of this height
    int group_rows[2];               // stepwise heights per kernel group (default or tuned)
    // Stepwise lattices form two groups, each stepped by its own launch: group 0 one
    // column per lane, group 1 two columns per lane (destination-scaled FP16, even
    // nx).  Group g holds dispatch positions [gfirst[g], gfirst[g] + gcount[g]) of
    // `desc` and `order`; its tile prefix sums start at tile_start + gfirst[g] + g and
    // its workgroup table at wg_first + wg_off[g].
    int gfirst[2], gcount[2], ntotal[2];
    size_t wg_off[2];
    int* tile_start;                 // device, n + 2 entries
    int* wg_first;                   // device, lattice of each workgroup's first tile
    size_t wg_capacity;              // entries available in wg_first
    hipGraph_t graph[2];
    hipGraphExec_t exec[2];
    hipEvent_t ev[2];                // bracket the last lb_batch_step (stepwise mode)
    std::vector<lb_ctx*> inst;       // per-lattice contexts on slices of the workspace
    std::vector<int> order;          // dispatch position -> lattice index
    std::vector<int> rows;           // strip height per lattice (current launch mode)
    lbmp::BatchInstance* desc;       // device descriptors in dispatch order
    unsigned long long* clocks;      // device, 2 per workgroup
    hipStream_t stream;
    int store, bc, psi;
    bool poisoned;
};

namespace {

// Whether lattice p is stepped two columns per lane in the stepwise batch.
bool batch_pair(const lb_params& p) { return lbmp::pair_step(p.store, p.nx); }

// Upper bound of the workgroups of the stepwise launches (one-row strips, one
// column per lane, the smallest workgroup), per group.
size_t batch_wg_capacity(const lb_params* p, int n)
{
    size_t tiles = 0;
    for (int i = 0; i < n; ++i) tiles += (size_t)((p[i].nx + lbmp::kTileW - 1) / lbmp::kTileW) * p[i].ny;
    const int wpb = std::min(lbmp::batch_waves_per_block(p[0].store, false), lbmp::batch_waves_per_block(p[0].store, true));
    return tiles / wpb + 4;
}

size_t batch_header_bytes(const lb_params* p, int n)
{
    return align_up((size_t)n * sizeof(lbmp::BatchInstance), kAlign) + align_up((size_t)n * 16, kAlign) +
           align_up((size_t)(n + 2) * sizeof(int), kAlign) + align_up(batch_wg_capacity(p, n) * sizeof(int), kAlign);
}

void drop_batch_graphs(lb_batch* b)
{
    for (int i = 0; i < 2; ++i) {
        if (b->exec[i]) (void)hipGraphExecDestroy(b->exec[i]);
        if (b->graph[i]) (void)hipGraphDestroy(b->graph[i]);
        b->exec[i] = nullptr;
        b->graph[i] = nullptr;
    }
}

// Dispatch order: in the stepwise mode the one-column lattices, then the
// two-column ones, each largest first (longest-processing-time order); in the
// persistent mode every lattice in one group (one column per lane), largest first.
void order_batch(lb_batch* b)
{
    const int n = b->n;
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    auto area = [&](int i) { return (long long)b->inst[i]->p.nx * b->inst[i]->p.ny; };
    auto grp = [&](int i) { return b->mode == LB_BATCH_STEPWISE && batch_pair(b->inst[i]->p) ? 1 : 0; };
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
        if (grp(x) != grp(y)) return grp(x) < grp(y);
        return area(x) > area(y);
    });
    b->order = idx;
    b->gcount[0] = b->gcount[1] = 0;
    for (int i = 0; i < n; ++i) ++b->gcount[grp(i)];
    b->gfirst[0] = 0;
    b->gfirst[1] = b->gcount[0];
}

// Strip height of lattice i in the current mode.
int lattice_rows(const lb_batch* b, int i)
{
    if (b->fixed_rows > 0) return b->fixed_rows;
    if (b->mode == LB_BATCH_PERSISTENT) return kBatchPersistentRows;
    return b->group_rows[batch_pair(b->inst[i]->p) ? 1 : 0];
}

// Copy the per-lattice launch descriptors (dispatch order) and the tile tables of
// both groups to the device.
hipError_t write_batch_descriptors(lb_batch* b)
{
    drop_batch_graphs(b);
    const int n = b->n;
    std::vector<lbmp::BatchInstance> host(n);
    std::vector<int> start(n + 2, 0);
    std::vector<int> first;
    b->rows.assign(n, 0);
    size_t woff = 0;
    for (int g = 0; g < 2; ++g) {
        const int j0 = b->gfirst[g], cnt = b->gcount[g];
        int* st = start.data() + j0 + g;
        st[0] = 0;
        for (int j = 0; j < cnt; ++j) {
            const int i = b->order[j0 + j];
            lb_ctx* c = b->inst[i];
            const int rows = lattice_rows(b, i);
            b->rows[i] = rows;
            lbmp::StepConst k = derive(c->p, rows, 1);
            if (g == 1) k.tiles_x = (c->p.nx + lbmp::kPairTileW - 1) / lbmp::kPairTileW;
            host[j0 + j].k = k;
            host[j0 + j].f[0] = c->f[0];
            host[j0 + j].f[1] = c->f[1];
            host[j0 + j].flag = c->flag;
            st[j + 1] = st[j] + k.tiles_x * k.tiles_y;
        }
        b->ntotal[g] = st[cnt];
        const int wpb = lbmp::batch_waves_per_block(b->store, g == 1);
        const int blocks = (b->ntotal[g] + wpb - 1) / wpb;
        b->wg_off[g] = woff;
        for (int blk = 0, i = 0; blk < blocks; ++blk) {
            const int t = blk * wpb;
            while (t >= st[i + 1]) ++i;
            first.push_back(i);
        }
        woff += (size_t)blocks;
    }
    if (woff > b->wg_capacity) return hipErrorInvalidValue;
    hipError_t e = hipMemcpyAsync(b->desc, host.data(), n * sizeof(lbmp::BatchInstance), hipMemcpyHostToDevice,
                                  b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->tile_start, start.data(), start.size() * sizeof(int), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && !first.empty())
        e = hipMemcpyAsync(b->wg_first, first.data(), first.size() * sizeof(int), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    return e;
}

// One step of every lattice (stepwise mode) reading buffer `parity`.
hipError_t batch_flat_launch(lb_batch* b, int parity)
{
    hipError_t e = hipSuccess;
    for (int g = 0; g < 2 && e == hipSuccess; ++g) {
        if (b->gcount[g] == 0) continue;
        e = lbmp::launch_batch_flat(b->store, b->bc == LB_BC_WALLS_Y, b->psi, g == 1, b->desc + b->gfirst[g],
                                    b->tile_start + b->gfirst[g] + g, b->wg_first + b->wg_off[g], b->ntotal[g],
                                    parity, b->stream);
    }
    return e;
}

lb_status build_batch_graph(lb_batch* b, int from)
{
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = hipSuccess;
    for (int i = 0; i < kDefaultGraphChunk && le == hipSuccess; ++i) le = batch_flat_launch(b, from ^ (i & 1));
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->stream, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(le, "batch launch during capture");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    b->graph[from] = g;
    b->exec[from] = x;
    return LB_OK;
}

lb_status validate_batch(const lb_params* p, int32_t n)
{
    if (!p || n < 1) return fail(LB_EINVAL, "need n >= 1 parameter blocks");
    for (int i = 0; i < n; ++i) {
        lb_status st = validate(p + i);
        if (st != LB_OK) return fail(st, "lattice " + std::to_string(i) + ": " + g_last_error);
        if (p[i].store != p[0].store || p[i].bc != p[0].bc || p[i].psi_form != p[0].psi_form)
            return fail(LB_EINVAL, "all lattices of a batch share store, bc and psi_form");
        if (p[i].stencil != LB_STENCIL_NEAREST)
            return fail(LB_EINVAL, "batched lattices use the nearest-neighbour stencil");
    }
    if (p[0].store != LB_STORE_F32 && p[0].store != LB_STORE_F16_LOCAL && p[0].store != LB_STORE_F16_DEST)
        return fail(LB_EINVAL, "batched storage must be LB_STORE_F32, LB_STORE_F16_LOCAL or LB_STORE_F16_DEST");
    return LB_OK;
}

}  // namespace

size_t lb_batch_workspace_bytes(const lb_params* p, int32_t n)
{
    if (validate_batch(p, n) != LB_OK) return 0;
    size_t total = batch_header_bytes(p, n);
    for (int i = 0; i < n; ++i) total += layout_of(p[i]).total;
    return total;
}

lb_status lb_batch_init(lb_batch** out, const lb_params* p, int32_t n, void* workspace,
                        size_t workspace_bytes, const float* const* rho0, const float* const* ux0,
                        const float* const* uy0, void* stream)
{
    if (!out) return fail(LB_EINVAL, "out is NULL");
    *out = nullptr;
    lb_status st = validate_batch(p, n);
    if (st != LB_OK) return st;
    if (!workspace || !rho0) return fail(LB_EINVAL, "workspace and rho0 must be non-NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(LB_EINVAL, "workspace must be 256-byte aligned");
    if (workspace_bytes < lb_batch_workspace_bytes(p, n))
        return fail(LB_ENOMEM, "workspace smaller than lb_batch_workspace_bytes");

    lb_batch* b = new (std::nothrow) lb_batch{};
    if (!b) return fail(LB_ENOMEM, "host allocation failed");
    b->n = n;
    b->stream = static_cast<hipStream_t>(stream);
    b->store = p[0].store;
    b->bc = p[0].bc;
    b->psi = p[0].psi_form;
    char* ws = static_cast<char*>(workspace);
    size_t hoff = 0;
    b->desc = reinterpret_cast<lbmp::BatchInstance*>(ws + hoff);
    hoff += align_up((size_t)n * sizeof(lbmp::BatchInstance), kAlign);
    b->clocks = reinterpret_cast<unsigned long long*>(ws + hoff);
    hoff += align_up((size_t)n * 16, kAlign);
    b->tile_start = reinterpret_cast<int*>(ws + hoff);
    hoff += align_up((size_t)(n + 2) * sizeof(int), kAlign);
    b->wg_first = reinterpret_cast<int*>(ws + hoff);
    b->wg_capacity = batch_wg_capacity(p, n);
    b->mode = LB_BATCH_STEPWISE;
    hipError_t ee = hipEventCreate(&b->ev[0]);
    if (ee == hipSuccess) ee = hipEventCreate(&b->ev[1]);
    if (ee != hipSuccess) {
        lb_batch_destroy(b);
        return hip_fail(ee, "hipEventCreate");
    }
    size_t off = batch_header_bytes(p, n);
    b->inst.assign(n, nullptr);
    for (int i = 0; i < n; ++i) {
        const size_t bytes = layout_of(p[i]).total;
        st = init_ctx(&b->inst[i], p + i, ws + off, bytes, rho0[i], ux0 ? ux0[i] : nullptr,
                      uy0 ? uy0[i] : nullptr, stream, false);
        if (st != LB_OK) {
            const std::string msg = g_last_error;
            lb_batch_destroy(b);
            return fail(st, "lattice " + std::to_string(i) + ": " + msg);
        }
        off += bytes;
    }
    b->group_rows[0] = b->group_rows[1] = default_batch_rows(b->store);
    order_batch(b);
    hipError_t e = write_batch_descriptors(b);
    if (e != hipSuccess) {
        lb_batch_destroy(b);
        return hip_fail(e, "batch descriptors");
    }
    for (int i = 0; i < n; ++i) {
        int hf = 0;
        st = read_flag(b->inst[i], &hf);
        if (st == LB_OK && (hf & lbmp::kFlagBadInput))
            st = fail(LB_EINVAL, "lattice " + std::to_string(i) + ": rho0/u0 out of range");
        if (st != LB_OK) {
            const std::string msg = g_last_error;
            lb_batch_destroy(b);
            return fail(st, msg);
        }
    }
    *out = b;
    g_last_error.clear();
    return LB_OK;
}

lb_status lb_batch_step(lb_batch* b, int64_t nsteps)
{
    if (!b) return fail(LB_EINVAL, "batch is NULL");
    if (b->poisoned) return fail(LB_ESTATE, "batch poisoned by an earlier failure");
    if (nsteps < 0 || nsteps > (1LL << 30)) return fail(LB_EINVAL, "nsteps must lie in [0, 2^30]");
    if (nsteps == 0) return LB_OK;
    int parity = b->inst[0]->cur;
    hipError_t e = hipSuccess;
    if (b->mode == LB_BATCH_PERSISTENT) {
        e = lbmp::launch_batch(b->store, b->bc == LB_BC_WALLS_Y, b->psi, b->desc, b->n, (int)nsteps, parity, b->clocks,
                               b->stream);
    } else {
        e = hipEventRecord(b->ev[0], b->stream);
        int64_t left = nsteps;
        while (e == hipSuccess && b->stream != nullptr && left >= kDefaultGraphChunk) {
            if (!b->exec[parity]) {
                lb_status st = build_batch_graph(b, parity);
                if (st != LB_OK) {
                    b->poisoned = true;
                    return st;
                }
            }
            e = hipGraphLaunch(b->exec[parity], b->stream);
            left -= kDefaultGraphChunk;  // even: the parity is unchanged
        }
        for (; e == hipSuccess && left > 0; --left) {
            e = batch_flat_launch(b, parity);
            parity ^= 1;
        }
        if (e == hipSuccess) e = hipEventRecord(b->ev[1], b->stream);
    }
    if (e != hipSuccess) {
        b->poisoned = true;
        return hip_fail(e, "batch launch");
    }
    for (lb_ctx* c : b->inst) {
        c->cur ^= (int)(nsteps & 1);
        c->t += nsteps;
    }
    return LB_OK;
}

static lb_ctx* batch_member(lb_batch* b, int32_t i)
{
    if (!b || i < 0 || i >= b->n) return nullptr;
    return b->inst[i];
}

lb_status lb_batch_moments(lb_batch* b, int32_t i, float* rho, float* ux, float* uy)
{
    lb_ctx* c = batch_member(b, i);
    if (!c) return fail(LB_EINVAL, "no such lattice");
    return lb_moments(c, rho, ux, uy);
}

lb_status lb_batch_diagnostics(lb_batch* b, int32_t i, const lb_region* in, const lb_region* outr, lb_diag* d)
{
    lb_ctx* c = batch_member(b, i);
    if (!c) return fail(LB_EINVAL, "no such lattice");
    return lb_diagnostics(c, in, outr, d);
}

lb_status lb_batch_diagnostics_all(lb_batch* b, const lb_region* in, const lb_region* outr, lb_diag* d)
{
    if (!b || !in || !outr || !d) return fail(LB_EINVAL, "NULL argument");
    if (b->poisoned) return fail(LB_ESTATE, "batch poisoned by an earlier failure");
    const int n = b->n;
    std::vector<double> h((size_t)n * lbmp::kDiagFields, 0.0);
    std::vector<int> hf(n, 0);
    hipError_t e = hipSuccess;
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        lb_ctx* c = b->inst[i];
        if (!c->poisoned)
            e = lbmp::launch_diag(c->p.store, c->p.bc == LB_BC_WALLS_Y, c->f[c->cur], c->kd, c->flag,
                                  diag_const(c, in + i, outr + i), c->partial, c->dout, b->stream);
    }
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        lb_ctx* c = b->inst[i];
        if (c->poisoned) continue;
        e = hipMemcpyAsync(&h[(size_t)i * lbmp::kDiagFields], c->dout, lbmp::kDiagFields * sizeof(double),
                           hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&hf[i], c->flag, sizeof(int), hipMemcpyDeviceToHost, b->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        b->poisoned = true;
        return hip_fail(e, "batch diagnostics");
    }
    int bad = 0;
    for (int i = 0; i < n; ++i) {
        lb_ctx* c = b->inst[i];
        fill_diag(c, &h[(size_t)i * lbmp::kDiagFields], hf[i], d + i);
        if (c->poisoned || d[i].unstable) {
            d[i].unstable = 1;
            c->poisoned = true;
            ++bad;
        }
    }
    return bad ? fail(LB_EUNSTABLE, std::to_string(bad) + " lattice(s) flagged an unstable site") : LB_OK;
}

lb_status lb_batch_get_state(lb_batch* b, int32_t i, void* dst)
{
    lb_ctx* c = batch_member(b, i);
    if (!c) return fail(LB_EINVAL, "no such lattice");
    return lb_get_state(c, dst);
}

lb_status lb_batch_check(lb_batch* b, int32_t* unstable)
{
    if (!b) return fail(LB_EINVAL, "batch is NULL");
    int count = 0;
    for (lb_ctx* c : b->inst) {
        int hf = 0;
        lb_status st = read_flag(c, &hf);
        if (st != LB_OK) return st;
        if (hf & lbmp::kFlagUnstable) {
            ++count;
            c->poisoned = true;
        }
    }
    if (unstable) *unstable = count;
    return count ? fail(LB_EUNSTABLE, std::to_string(count) + " lattice(s) flagged an unstable site") : LB_OK;
}

lb_status lb_batch_times(lb_batch* b, double* seconds)
{
    if (!b || !seconds) return fail(LB_EINVAL, "NULL argument");
    if (b->mode == LB_BATCH_STEPWISE) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(b->ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, b->ev[0], b->ev[1]);
        if (e != hipSuccess) return hip_fail(e, "batch events");
        for (int i = 0; i < b->n; ++i) seconds[i] = ms * 1e-3;
        return LB_OK;
    }
    std::vector<unsigned long long> h(2 * (size_t)b->n);
    hipError_t e = hipMemcpyAsync(h.data(), b->clocks, h.size() * sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    int dev = 0, khz = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return hip_fail(e, "batch clocks");
    if (khz <= 0) return fail(LB_EHIP, "device reports no wall-clock rate");
    unsigned long long t0 = h[0];
    for (int j = 0; j < b->n; ++j) t0 = std::min(t0, h[2 * j]);
    for (int j = 0; j < b->n; ++j) seconds[b->order[j]] = (double)(h[2 * j + 1] - t0) / (khz * 1e3);
    return LB_OK;
}

lb_status lb_batch_set_launch(lb_batch* b, int32_t mode, int32_t strip_rows)
{
    if (!b) return fail(LB_EINVAL, "batch is NULL");
    if (mode != LB_BATCH_STEPWISE && mode != LB_BATCH_PERSISTENT) return fail(LB_EINVAL, "unknown batch mode");
    if (strip_rows < 0 || strip_rows > kMaxStripRows) return fail(LB_EINVAL, "strip_rows must lie in [0, 64]");
    b->mode = mode;
    b->fixed_rows = strip_rows;
    order_batch(b);
    hipError_t e = write_batch_descriptors(b);
    if (e != hipSuccess) return hip_fail(e, "batch descriptors");
    return LB_OK;
}

lb_status lb_batch_tune(lb_batch* b, int32_t trial_steps, int32_t* rows_out)
{
    if (!b) return fail(LB_EINVAL, "batch is NULL");
    if (b->poisoned) return fail(LB_ESTATE, "batch poisoned by an earlier failure");
    if (trial_steps < 1 || trial_steps > 1000) return fail(LB_EINVAL, "trial_steps must lie in [1, 1000]");
    if (b->mode != LB_BATCH_STEPWISE) return fail(LB_EINVAL, "lb_batch_tune tunes the stepwise mode");
    if (b->stream == nullptr) return fail(LB_EINVAL, "lb_batch_tune needs a stream other than the legacy stream");
    b->fixed_rows = 0;
    const int parity = b->inst[0]->cur;
    // Seconds of `trial_steps` launches that all read buffer `parity` and write the
    // other one: the state (buffer parity) is unchanged, and the other buffer is
    // overwritten in full by the next step.  The least of three repetitions.
    auto time_launches = [&](double& sec) -> hipError_t {
        hipError_t e = write_batch_descriptors(b);
        for (int w = 0; w < 2 && e == hipSuccess; ++w) e = batch_flat_launch(b, parity);
        sec = 1e30;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            e = hipEventRecord(b->ev[0], b->stream);
            for (int t = 0; t < trial_steps && e == hipSuccess; ++t) e = batch_flat_launch(b, parity);
            if (e == hipSuccess) e = hipEventRecord(b->ev[1], b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(b->ev[1]);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, b->ev[0], b->ev[1]);
            sec = std::min(sec, ms * 1e-3);
        }
        return e;
    };
    // each kernel group (the larger first) gets the height that runs its share of the
    // batch fastest, with the other group at its current height
    const int first = b->gcount[1] > b->gcount[0] ? 1 : 0;
    for (int gi = 0; gi < 2; ++gi) {
        const int g = gi == 0 ? first : 1 - first;
        if (b->gcount[g] == 0) continue;
        int best_r = b->group_rows[g];
        double best = 1e30;
        hipError_t e = hipSuccess;
        for (int cand = 1; cand <= kTuneMaxRows && e == hipSuccess; ++cand) {
            b->group_rows[g] = cand;
            double sec = 0.0;
            e = time_launches(sec);
            if (e == hipSuccess && sec < best) {
                best = sec;
                best_r = cand;
            }
        }
        b->group_rows[g] = best_r;
        if (e != hipSuccess) {
            b->poisoned = true;
            return hip_fail(e, "lb_batch_tune trial launches");
        }
    }
    hipError_t e = write_batch_descriptors(b);
    if (e != hipSuccess) return hip_fail(e, "batch descriptors");
    if (rows_out)
        for (int i = 0; i < b->n; ++i) rows_out[i] = b->rows[i];
    return LB_OK;
}

lb_status lb_batch_destroy(lb_batch* b)
{
    if (!b) return LB_OK;
    drop_batch_graphs(b);
    for (int i = 0; i < 2; ++i)
        if (b->ev[i]) (void)hipEventDestroy(b->ev[i]);
    for (lb_ctx* c : b->inst)
        if (c) lb_destroy(c);
    delete b;
    return LB_OK;
}

lb_status lb_copy_probe(const void* src, void* dst, size_t bytes, void* stream)
{
    if (!src || !dst || bytes % 16) return fail(LB_EINVAL, "need non-NULL buffers and bytes % 16 == 0");
    hipError_t e = lbmp::launch_copy_probe(src, dst, (long long)(bytes / 16), static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "copy probe launch");
    return LB_OK;
}

}  // extern "C"
