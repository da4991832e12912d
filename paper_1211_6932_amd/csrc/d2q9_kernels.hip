// d2q9_kernels.hip -- gfx950 kernels of the improved MRT pseudopotential D2Q9
// method and their host-side launchers.
//
//   d2q9_strip<store, walls, MODE, psi form>
//                     one template walks a wavefront strip (pull, density,
//                     psi of Eq. (24) or Eq. (23), force, velocity) and then, by
//                     MODE, collides and stores (the time step), writes rho/v
//                     (moments), or accumulates FP64 reductions (diagnostics).
//   d2q9_pair<walls, psi form>
//                     the time step of the destination-scaled FP16 storage
//                     with two columns per lane (even nx), bitwise the same
//                     as d2q9_strip's
//   d2q9_batch        persistent multi-instance step (one workgroup per lattice)
//   d2q9_batch_flat   one step of many lattices in one launch over their strips
//   d2q9_init         equilibrium initial state, written "pre-streamed" so
//                     that the first pull returns f_eq(rho0, u0)
//   diag_finalize     fixed-order FP64 reduction of the per-wave partials
//   copy_probe        plain streaming copy: attainable-bandwidth reference
#include "d2q9_core.hpp"
#include "d2q9_launch.hpp"

namespace lbmp {


// Wave priorities (s_setprio) while a wavefront issues loads: the prologue of a
// strip (its first rows) above the prefetch of the next row inside the walk,
// both above everything else (arithmetic and stores).  A wave that has just
// started then gets its first requests out ahead of the resident waves, and
// those issue their prefetches ahead of other waves' arithmetic.  Measured on
// the 8192 x 4096 splash, FP32: 78.6k MLUPS against 76.1k without priorities,
// 77.4k with the prologue raised alone and 77.4k with both raised to the same
// level.
constexpr short kPrioPrologue = 2;
constexpr short kPrioPrefetch = 1;


// rho and the Eq. (6) velocity of site (xci, y) into the [ny][nx] output fields.
__device__ __forceinline__ void write_moments(const StepConst& k, int y, int xci, float r, float vx, float vy,
                                              float* __restrict__ rho_out, float* __restrict__ ux_out,
                                              float* __restrict__ uy_out)
{
    const long long o = (long long)y * k.nx + xci;
    if (rho_out) rho_out[o] = r;
    if (ux_out) ux_out[o] = vx;
    if (uy_out) uy_out[o] = vy;
}

// FP64 diagnostics of one site: mass, momentum, pressure (Eq. 30 or the Eq. (23)
// bulk pressure) and density sums over the two annuli, max |v|.
__device__ __forceinline__ void diag_accumulate(const StepConst& k, const DiagConst& dg, int y, int xci, float r,
                                                float vx, float vy, double acc[kDiagFields])
{
    const double rr = r;
    const double pr = pressure_f64(rr, dg.psi);
    acc[0] += rr;
    acc[1] += rr * (double)vx;
    acc[2] += rr * (double)vy;
    double dx = fabs((double)xci - dg.in_cx);
    dx = fmin(dx, (double)k.nx - dx);
    double dy = fabs((double)y - dg.in_cy);
    if (dg.periodic_y) dy = fmin(dy, (double)k.ny - dy);
    double d = sqrt(dx * dx + dy * dy);
    if (d >= dg.in_r0 && d < dg.in_r1) { acc[3] += pr; acc[5] += rr; acc[7] += 1.0; }
    dx = fabs((double)xci - dg.out_cx);
    dx = fmin(dx, (double)k.nx - dx);
    dy = fabs((double)y - dg.out_cy);
    if (dg.periodic_y) dy = fmin(dy, (double)k.ny - dy);
    d = sqrt(dx * dx + dy * dy);
    if (d >= dg.out_r0 && d < dg.out_r1) { acc[4] += pr; acc[6] += rr; acc[8] += 1.0; }
    acc[9] = fmax(acc[9], (double)sqrtf(vx * vx + vy * vy));
}

// Wave-reduce the per-lane diagnostics and write the wave's partial for `tile`.
__device__ __forceinline__ void diag_write(double acc[kDiagFields], int lane, int tile, double* __restrict__ partial)
{
    for (int i = 0; i < 9; ++i) acc[i] = wave_sum(acc[i]);
    acc[9] = wave_max(acc[9]);
    if (lane == 0) {
        for (int i = 0; i < kDiagFields; ++i) partial[(long long)tile * kDiagFields + i] = acc[i];
    }
}

// One wavefront walks the rows of its strip in direction DIR (+1: y0 up to
// y1 - 1; -1: y1 - 1 down to y0).  Every row is pulled and reduced to density and
// psi once; the force at a row needs psi of the rows on both sides, so the walk
// starts with the row just outside the strip on its entry side and also pulls
// the row just outside on its exit side.  Each site's arithmetic is the same in
// both directions, so the results are bitwise independent of DIR.
template <int S, bool WALLS, int MODE, int PSI, int DIR>
__device__ __forceinline__ void strip_walk(
    const typename Codec<S>::T* __restrict__ fin, typename Codec<S>::T* __restrict__ fout,
    const StepConst& k, const int tile, const int lane, const int ty, const bool live, const int xci,
    const unsigned xm, const unsigned xc, const unsigned xp, int* __restrict__ flag,
    float* __restrict__ rho_out, float* __restrict__ ux_out, float* __restrict__ uy_out,
    const DiagConst& dg, double* __restrict__ partial)
{
    using C = Codec<S>;
    static_assert(DIR == 1 || DIR == -1, "walk direction");
    const int y0 = ty * k.strip_rows;
    const int y1 = min(y0 + k.strip_rows, k.ny);
    const int n = y1 - y0;
    const int ys = DIR > 0 ? y0 : y1 - 1;  // first row walked

    // row y is present in the lattice (walls) or wraps (periodic)
    auto inside = [&](const int y) __attribute__((always_inline)) { return !WALLS || (y >= 0 && y < k.ny); };
    auto wrap = [&](const int y) __attribute__((always_inline)) {
        return y < 0 ? y + k.ny : (y >= k.ny ? y - k.ny : y);
    };

    bool bad = false;
    // Three row buffers (rows y, y+DIR, y+2 DIR in flight), three psi windows and
    // three windows of 1/rhohat (destination-scaled storage) for rows y-DIR, y,
    // y+DIR, each a value and its two x-neighbours, and three densities.  The row
    // loop below is unrolled three times with the roles rotated, so sliding the
    // window along the strip moves no data.
    struct Win { float L, C, R; };
    float fa[9], fb[9], fc[9];
    Win wa{0.0f, 0.0f, 0.0f}, wb{0.0f, 0.0f, 0.0f}, wc{0.0f, 0.0f, 0.0f};
    Win ia{0.0f, 0.0f, 0.0f}, ib{0.0f, 0.0f, 0.0f}, ic{0.0f, 0.0f, 0.0f};
    float ra = 0.0f, rb = 0.0f, rc = 0.0f;

    // psi of the row before the first one walked, or its mirror at a wall
    float pm = 0.0f, im = 0.0f;
    const int yh = ys - DIR;
    const bool has_h = inside(yh);
    __builtin_amdgcn_s_setprio(kPrioPrologue);
    if (has_h) {
        pull_row<S, WALLS>(fin, k, wrap(yh), xm, xc, xp, fb);
        const float rm = density(fb);
        pm = pseudopotential<PSI>(rm, k, bad);
        if constexpr (C::kDestScaled) im = recip(C::round_scale(rm));
    }
    pull_row<S, WALLS>(fin, k, ys, xm, xc, xp, fa);
    // the second row is requested before the first is consumed (two rows in flight)
    if (inside(ys + DIR)) pull_row<S, WALLS>(fin, k, wrap(ys + DIR), xm, xc, xp, fb);
    __builtin_amdgcn_s_setprio(0);
    ra = density(fa);
    const float pc0 = pseudopotential<PSI>(ra, k, bad);
    if (!has_h) pm = pc0;
    wa = Win{lane_from_left(pm), pm, lane_from_right(pm)};
    wb = Win{lane_from_left(pc0), pc0, lane_from_right(pc0)};
    if constexpr (C::kDestScaled) {
        const float ic0 = recip(C::round_scale(ra));
        if (!has_h) im = ic0;
        ia = Win{lane_from_left(im), im, lane_from_right(im)};
        ib = Win{lane_from_left(ic0), ic0, lane_from_right(ic0)};
    }

    double acc[kDiagFields];
    if (MODE == kModeDiag) {
        for (int i = 0; i < kDiagFields; ++i) acc[i] = 0.0;
    }

    // Row y at walk position i.  f: row y (pulled), fn: row y+DIR (pulled), fq:
    // receives row y+2 DIR; r: density of row y, rn: receives the density of row
    // y+DIR; psi windows b, c (rows y-DIR, y) and a (receives row y+DIR); likewise
    // the 1/rhohat windows.
    auto row = [&](const int i, float (&f)[9], float (&fn)[9], float (&fq)[9], float& r, float& rn,
                   const Win& b, const Win& c, Win& a, const Win& db, const Win& dc, Win& da)
                   __attribute__((always_inline)) {
        const int y = ys + DIR * i;
        const bool has_n = inside(y + DIR);
        // rows up to one beyond the strip's last are pulled
        __builtin_amdgcn_s_setprio(kPrioPrefetch);
        if (i + 2 <= n && inside(y + 2 * DIR)) pull_row<S, WALLS>(fin, k, wrap(y + 2 * DIR), xm, xc, xp, fq);
        __builtin_amdgcn_s_setprio(0);
        float pa;
        rn = 0.0f;
        if (has_n) {
            rn = density(fn);
            pa = pseudopotential<PSI>(rn, k, bad);
        } else {
            pa = c.C;  // mirror beyond a wall
        }
        a = Win{lane_from_left(pa), pa, lane_from_right(pa)};
        if constexpr (C::kDestScaled) {
            const float in = has_n ? recip(C::round_scale(rn)) : dc.C;
            da = Win{lane_from_left(in), in, lane_from_right(in)};
        }
        // windows of rows y - 1 and y + 1
        const Win& m = DIR > 0 ? b : a;
        const Win& p = DIR > 0 ? a : b;
        const Win& dm = DIR > 0 ? db : da;
        const Win& dp = DIR > 0 ? da : db;

        float Fx, Fy, Fs2;
        force_stencil(m.L, m.C, m.R, c.L, c.C, c.R, p.L, p.C, p.R, k, Fx, Fy, Fs2);
        const float jx = (f[1] - f[3]) + ((f[5] - f[7]) + (f[8] - f[6]));
        const float jy = (f[2] - f[4]) + ((f[5] - f[7]) + (f[6] - f[8]));
        const float inv_rho = recip(r);
        const float vx = fmaf(0.5f, Fx, jx) * inv_rho;
        const float vy = fmaf(0.5f, Fy, jy) * inv_rho;

        if (MODE == kModeStep) {
            collide(f, r, vx, vy, Fx, Fy, Fs2, k);
            if (live) {
                typename C::T* out = fout + (long long)y * k.row_stride;
                if constexpr (C::kDestScaled) {
                    // 1/rhohat of the site that pulls population a next step: the
                    // neighbour at x + e_a, or this site for a population that
                    // reflects at a wall
                    const bool bot = WALLS && y == 0, top = WALLS && y == k.ny - 1;
                    float id[9];
                    id[0] = dc.C;
                    id[1] = dc.R;
                    id[3] = dc.L;
                    id[2] = top ? dc.C : dp.C;
                    id[5] = top ? dc.C : dp.R;
                    id[6] = top ? dc.C : dp.L;
                    id[4] = bot ? dc.C : dm.C;
                    id[7] = bot ? dc.C : dm.L;
                    id[8] = bot ? dc.C : dm.R;
#pragma unroll
                    for (int a = 0; a < 9; ++a) C::store(out, k, a, xc, f[a], id[a]);
                } else {
#pragma unroll
                    for (int a = 0; a < 9; ++a) C::store(out, k, a, xc, f[a], inv_rho);
                }
                C::store_density(out, k, xc, r);
            }
        } else if (MODE == kModeMoments) {
            if (live) write_moments(k, y, xci, r, vx, vy, rho_out, ux_out, uy_out);
        } else {
            if (live) diag_accumulate(k, dg, y, xci, r, vx, vy, acc);
        }
    };

    for (int i = 0; i < n; i += 3) {
        row(i, fa, fb, fc, ra, rb, wa, wb, wc, ia, ib, ic);
        if (i + 1 >= n) break;
        row(i + 1, fb, fc, fa, rb, rc, wb, wc, wa, ib, ic, ia);
        if (i + 2 >= n) break;
        row(i + 2, fc, fa, fb, rc, ra, wc, wa, wb, ic, ia, ib);
    }

    if (MODE == kModeDiag) diag_write(acc, lane, tile, partial);
    if (bad) flag[0] = kFlagUnstable;  // vector store from any flagging lane; all write the same value
}

// One wavefront processes strip `tile` of the lattice described by `k`: pull,
// density, psi, force and velocity for every row, then by MODE collide and
// store (a time step), write rho/v (moments) or accumulate FP64 reductions.
template <int S, bool WALLS, int MODE, int PSI>
__device__ __forceinline__ void strip_tile(
    const typename Codec<S>::T* __restrict__ fin, typename Codec<S>::T* __restrict__ fout,
    const StepConst& k, const int tile, const int lane, int* __restrict__ flag,
    float* __restrict__ rho_out, float* __restrict__ ux_out, float* __restrict__ uy_out,
    const DiagConst& dg, double* __restrict__ partial)
{
    using C = Codec<S>;
    // Tiles are numbered in bands of `band` strips: within a band, consecutive
    // tiles go down the strips first, so the wavefronts of one workgroup cover a
    // small rectangle and share halo rows and columns in the CU's L1.
    const int band0 = (tile / (k.tiles_x * k.band)) * k.band;
    const int band_h = min(k.band, k.tiles_y - band0);
    const int r = tile - band0 * k.tiles_x;
    const int tx = r / band_h;
    const int ty = band0 + r % band_h;

    // Column of this lane; lanes 0 and 63 are the psi halo.  Columns wrap in x.
    const int xs = tx * kTileW - 1 + lane;
    const bool live = (lane >= 1) && (lane <= kTileW) && (xs < k.nx);
    int xci = xs < 0 ? xs + k.nx : (xs >= k.nx ? xs - k.nx : xs);
    if (xs > k.nx) xci = 0;  // beyond the right halo: in-range dummy column, never stored
    // byte offsets of columns x, x-1, x+1 within a row
    const unsigned eb = sizeof(typename C::T);
    const unsigned xc = (unsigned)xci * eb;
    const unsigned xm = (unsigned)((xci == 0) ? k.nx - 1 : xci - 1) * eb;
    const unsigned xp = (unsigned)((xci == k.nx - 1) ? 0 : xci + 1) * eb;

    // In a time step of a 16-bit encoding, strips of odd index walk towards
    // decreasing y and the others towards increasing y: two strips that share a
    // boundary then reach the rows on both sides of it at about the same point of
    // their walks.  (Neighbouring strips start at about the same time; walking the
    // same way, one would read the shared rows at the start and the other at the
    // end of its walk.)  Measured on the 8192 x 4096 splash: +3 % for global FP16
    // offsets, +0.4 % for destination-scaled FP16, and -5 % for FP32, which keeps
    // one direction.
    constexpr bool alt = sizeof(typename C::T) == 2;
    if constexpr (MODE == kModeStep && alt) {
        if (ty & 1) {
            strip_walk<S, WALLS, MODE, PSI, -1>(fin, fout, k, tile, lane, ty, live, xci, xm, xc, xp, flag,
                                                rho_out, ux_out, uy_out, dg, partial);
            return;
        }
    }
    strip_walk<S, WALLS, MODE, PSI, 1>(fin, fout, k, tile, lane, ty, live, xci, xm, xc, xp, flag, rho_out,
                                       ux_out, uy_out, dg, partial);
}

template <int S, bool WALLS, int MODE, int PSI>
__global__ __launch_bounds__(kWave * step_waves_per_block(S))
__attribute__((amdgpu_waves_per_eu(1))) void d2q9_strip(
    const typename Codec<S>::T* __restrict__ fin, typename Codec<S>::T* __restrict__ fout,
    StepConst k, int* __restrict__ flag, float* __restrict__ rho_out, float* __restrict__ ux_out,
    float* __restrict__ uy_out, DiagConst dg, double* __restrict__ partial)
{
    const int lane = threadIdx.x & (kWave - 1);
    // the wave index is uniform across the wave: keep it (and every row address
    // derived from it) in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = logical_block(blockIdx.x, gridDim.x) * step_waves_per_block(S) + wave;
    if (tile >= k.tiles_x * k.tiles_y) return;  // whole wavefront leaves together
    strip_tile<S, WALLS, MODE, PSI>(fin, fout, k, tile, lane, flag, rho_out, ux_out, uy_out, dg, partial);
}

// ---------------------------------------------------------------- two columns per lane
// Time step of the destination-scaled FP16 storage with two neighbouring
// columns per lane.  The 16-bit step is bound by the number of vector memory
// instructions, not by bytes: one 16-bit element per lane moves 128 bytes per
// instruction.  Here every access is an aligned 32-bit pair (256 bytes per
// instruction, half the instructions per site), and the one-column shift of the
// pull along x comes from the neighbouring lane's pair (a lane shuffle) instead
// of an unaligned load.  A wavefront covers 128 columns: lanes 1..62 own the 124
// output columns, lane 0's second column and the first column right of the
// output are the psi halo.  Each site's arithmetic is that of strip_walk, so the
// results are bitwise those of the one-column kernel.  Needs an even nx, so that
// no pair straddles the periodic seam.

__device__ __forceinline__ float f16_lo(unsigned w)
{
    return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<unsigned short>(w & 0xffffu)));
}
__device__ __forceinline__ float f16_hi(unsigned w)
{
    return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<unsigned short>(w >> 16)));
}
__device__ __forceinline__ float bf16_lo(unsigned w)
{
    return static_cast<float>(__builtin_bit_cast(__bf16, static_cast<unsigned short>(w & 0xffffu)));
}
__device__ __forceinline__ float bf16_hi(unsigned w)
{
    return static_cast<float>(__builtin_bit_cast(__bf16, static_cast<unsigned short>(w >> 16)));
}
// Two FP16 values (round to nearest even) in one 32-bit word, low half first.  Built
// as a two-element vector so that the conversions write the two halves of one
// register directly (no separate or/shift to pack them).
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned pack_f16(float lo, float hi)
{
    const half2v v = {static_cast<_Float16>(lo), static_cast<_Float16>(hi)};
    return __builtin_bit_cast(unsigned, v);
}
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned pack_bf16(float lo, float hi)
{
    const bf16x2v v = {static_cast<__bf16>(lo), static_cast<__bf16>(hi)};
    return __builtin_bit_cast(unsigned, v);
}

// Raw pairs of lattice row y for the pull (Eq. 5): w[a] holds population a's
// pair from the row it streams from (the row itself for a population that
// reflects at a wall), w[9] the row's own bf16 scale pair.  qb: byte offset of
// the lane's pair within a row.
template <bool WALLS>
__device__ __forceinline__ void pull_pair(const _Float16* __restrict__ fin, const StepConst& k, int y,
                                          unsigned qb, unsigned w[10])
{
    int ya = y - 1, yb = y + 1;
    bool bot = false, top = false;
    if (WALLS) {
        bot = ya < 0;
        top = yb >= k.ny;
    } else {
        if (ya < 0) ya += k.ny;
        if (yb >= k.ny) yb -= k.ny;
    }
    const _Float16* r0 = fin + (long long)y * k.row_stride;
    const _Float16* ra = fin + (long long)(bot ? y : ya) * k.row_stride;
    const _Float16* rb = fin + (long long)(top ? y : yb) * k.row_stride;
    using T = _Float16;
    w[0] = ld<unsigned>(r0, slot_bytes<T>(k, 0), qb);
    w[1] = ld<unsigned>(r0, slot_bytes<T>(k, 1), qb);
    w[3] = ld<unsigned>(r0, slot_bytes<T>(k, 3), qb);
    w[2] = ld<unsigned>(ra, slot_bytes<T>(k, bot ? 4 : 2), qb);
    w[5] = ld<unsigned>(ra, slot_bytes<T>(k, bot ? 7 : 5), qb);
    w[6] = ld<unsigned>(ra, slot_bytes<T>(k, bot ? 8 : 6), qb);
    w[4] = ld<unsigned>(rb, slot_bytes<T>(k, top ? 2 : 4), qb);
    w[7] = ld<unsigned>(rb, slot_bytes<T>(k, top ? 5 : 7), qb);
    w[8] = ld<unsigned>(rb, slot_bytes<T>(k, top ? 6 : 8), qb);
    w[9] = ld<unsigned>(r0, slot_bytes<T>(k, 9), qb);
}

// Pulled populations of the lane's two sites (f0: left column, f1: right
// column) from the raw pairs of row y.  A population moving in +x comes from
// the column on the left: the high half of the left lane's pair for the first
// site, the low half of the own pair for the second; one moving in -x from the
// right; a population that reflects at a wall from the own column.
template <bool WALLS>
__device__ __forceinline__ void decode_pair(const StepConst& k, int y, const unsigned w[10], float f0[9],
                                            float f1[9])
{
    const bool bot = WALLS && y == 0, top = WALLS && y == k.ny - 1;
    const unsigned l1 = __shfl_up(w[1], 1, kWave), l5 = __shfl_up(w[5], 1, kWave);
    const unsigned l8 = __shfl_up(w[8], 1, kWave);
    const unsigned r3 = __shfl_down(w[3], 1, kWave), r6 = __shfl_down(w[6], 1, kWave);
    const unsigned r7 = __shfl_down(w[7], 1, kWave);
    f0[0] = f16_lo(w[0]); f1[0] = f16_hi(w[0]);
    f0[2] = f16_lo(w[2]); f1[2] = f16_hi(w[2]);
    f0[4] = f16_lo(w[4]); f1[4] = f16_hi(w[4]);
    f0[1] = f16_hi(l1);   f1[1] = f16_lo(w[1]);
    f0[3] = f16_hi(w[3]); f1[3] = f16_lo(r3);
    f0[5] = bot ? f16_lo(w[5]) : f16_hi(l5);
    f1[5] = bot ? f16_hi(w[5]) : f16_lo(w[5]);
    f0[6] = bot ? f16_lo(w[6]) : f16_hi(w[6]);
    f1[6] = bot ? f16_hi(w[6]) : f16_lo(r6);
    f0[7] = top ? f16_lo(w[7]) : f16_hi(w[7]);
    f1[7] = top ? f16_hi(w[7]) : f16_lo(r7);
    f0[8] = top ? f16_lo(w[8]) : f16_hi(l8);
    f1[8] = top ? f16_hi(w[8]) : f16_lo(w[8]);
    // f_a = rhohat (w_a + g_a) with the puller's own scale (as pull_row)
    const float sc[2] = {bf16_lo(w[9]), bf16_hi(w[9])};
    float* f[2] = {f0, f1};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const float sw0 = sc[j] * (4.0f / 9.0f), sw1 = sc[j] * (1.0f / 9.0f), sw2 = sc[j] * (1.0f / 36.0f);
        f[j][0] = fmaf(f[j][0], sc[j], sw0);
#pragma unroll
        for (int a = 1; a < 5; ++a) f[j][a] = fmaf(f[j][a], sc[j], sw1);
#pragma unroll
        for (int a = 5; a < 9; ++a) f[j][a] = fmaf(f[j][a], sc[j], sw2);
    }
}

// Values of a row at the lane's two sites and at the sites next to them: s0, s1
// (own), L (left lane's second site), R (right lane's first site).
struct PairWin { float s0, s1, L, R; };
__device__ __forceinline__ PairWin pair_window(float v0, float v1)
{
    return PairWin{v0, v1, lane_from_left(v1), lane_from_right(v0)};
}

template <bool WALLS, int PSI, int DIR>
__device__ __forceinline__ void pair_walk(const _Float16* __restrict__ fin, _Float16* __restrict__ fout,
                                          const StepConst& k, const int ty, const bool live, const unsigned qb,
                                          int* __restrict__ flag)
{
    using C = Codec<kStoreF16Dest>;
    const int y0 = ty * k.strip_rows;
    const int y1 = min(y0 + k.strip_rows, k.ny);
    const int n = y1 - y0;
    const int ys = DIR > 0 ? y0 : y1 - 1;
    auto inside = [&](const int y) __attribute__((always_inline)) { return !WALLS || (y >= 0 && y < k.ny); };
    auto wrap = [&](const int y) __attribute__((always_inline)) {
        return y < 0 ? y + k.ny : (y >= k.ny ? y - k.ny : y);
    };
    // the unstable flag counts output sites only (every site is an output site of one lane)
    bool bad = false;
    auto psi2 = [&](const float r0, const float r1, float& p0, float& p1) __attribute__((always_inline)) {
        bool b = false;
        p0 = pseudopotential<PSI>(r0, k, b);
        p1 = pseudopotential<PSI>(r1, k, b);
        bad = bad || (b && live);
    };

    float fa0[9], fa1[9], fb0[9], fb1[9];
    unsigned wa[10], wb[10];
    PairWin pm, pc, im, ic;
    float ra0, ra1;

    // row before the first one walked (or its mirror at a wall), then the first
    // two rows in flight
    const int yh = ys - DIR;
    const bool has_h = inside(yh);
    __builtin_amdgcn_s_setprio(kPrioPrologue);
    float h0 = 0.0f, h1 = 0.0f, hi0 = 0.0f, hi1 = 0.0f;
    if (has_h) {
        pull_pair<WALLS>(fin, k, wrap(yh), qb, wa);
        decode_pair<WALLS>(k, wrap(yh), wa, fb0, fb1);
        const float rm0 = density(fb0), rm1 = density(fb1);
        psi2(rm0, rm1, h0, h1);
        hi0 = recip(C::round_scale(rm0));
        hi1 = recip(C::round_scale(rm1));
    }
    pull_pair<WALLS>(fin, k, ys, qb, wa);
    if (inside(ys + DIR)) pull_pair<WALLS>(fin, k, wrap(ys + DIR), qb, wb);
    __builtin_amdgcn_s_setprio(0);
    decode_pair<WALLS>(k, ys, wa, fa0, fa1);
    ra0 = density(fa0);
    ra1 = density(fa1);
    float c0, c1;
    psi2(ra0, ra1, c0, c1);
    const float ci0 = recip(C::round_scale(ra0)), ci1 = recip(C::round_scale(ra1));
    if (!has_h) {
        h0 = c0; h1 = c1;
        hi0 = ci0; hi1 = ci1;
    }
    pm = pair_window(h0, h1);
    pc = pair_window(c0, c1);
    im = pair_window(hi0, hi1);
    ic = pair_window(ci0, ci1);

    // Row y at walk position i: f (decoded row y) and its densities r; wn holds
    // the raw pairs of row y+DIR, wq receives those of row y+2 DIR; g receives
    // the decoded row y+DIR.  Windows b, c: psi of rows y-DIR, y (likewise the
    // 1/rhohat windows db, dc); on return b, db hold row y+DIR's windows
    // (c, dc are left for the caller to rotate).
    auto row = [&](const int i, float (&f0)[9], float (&f1)[9], float& r0, float& r1, float (&g0)[9],
                   float (&g1)[9], const unsigned (&wn)[10], unsigned (&wq)[10], PairWin& b, const PairWin& c,
                   PairWin& db, const PairWin& dc) __attribute__((always_inline)) {
        const int y = ys + DIR * i;
        const bool has_n = inside(y + DIR);
        float rn0 = 0.0f, rn1 = 0.0f, pa0, pa1, in0, in1;
        if (has_n) decode_pair<WALLS>(k, wrap(y + DIR), wn, g0, g1);
        __builtin_amdgcn_s_setprio(kPrioPrefetch);
        if (i + 2 <= n && inside(y + 2 * DIR)) pull_pair<WALLS>(fin, k, wrap(y + 2 * DIR), qb, wq);
        __builtin_amdgcn_s_setprio(0);
        if (has_n) {
            rn0 = density(g0);
            rn1 = density(g1);
            psi2(rn0, rn1, pa0, pa1);
            in0 = recip(C::round_scale(rn0));
            in1 = recip(C::round_scale(rn1));
        } else {  // mirror beyond a wall
            pa0 = c.s0; pa1 = c.s1;
            in0 = dc.s0; in1 = dc.s1;
        }
        const PairWin a = pair_window(pa0, pa1);
        const PairWin da = pair_window(in0, in1);
        // windows of rows y - 1 and y + 1
        const PairWin& m = DIR > 0 ? b : a;
        const PairWin& p = DIR > 0 ? a : b;
        const PairWin& dm = DIR > 0 ? db : da;
        const PairWin& dp = DIR > 0 ? da : db;

        float Fx0, Fy0, Fs20, Fx1, Fy1, Fs21;
        force_stencil(m.L, m.s0, m.s1, c.L, c.s0, c.s1, p.L, p.s0, p.s1, k, Fx0, Fy0, Fs20);
        force_stencil(m.s0, m.s1, m.R, c.s0, c.s1, c.R, p.s0, p.s1, p.R, k, Fx1, Fy1, Fs21);
        {
            const float jx = (f0[1] - f0[3]) + ((f0[5] - f0[7]) + (f0[8] - f0[6]));
            const float jy = (f0[2] - f0[4]) + ((f0[5] - f0[7]) + (f0[6] - f0[8]));
            const float inv_rho = recip(r0);
            collide(f0, r0, fmaf(0.5f, Fx0, jx) * inv_rho, fmaf(0.5f, Fy0, jy) * inv_rho, Fx0, Fy0, Fs20, k);
        }
        {
            const float jx = (f1[1] - f1[3]) + ((f1[5] - f1[7]) + (f1[8] - f1[6]));
            const float jy = (f1[2] - f1[4]) + ((f1[5] - f1[7]) + (f1[6] - f1[8]));
            const float inv_rho = recip(r1);
            collide(f1, r1, fmaf(0.5f, Fx1, jx) * inv_rho, fmaf(0.5f, Fy1, jy) * inv_rho, Fx1, Fy1, Fs21, k);
        }
        if (live) {
            _Float16* out = fout + (long long)y * k.row_stride;
            // 1/rhohat of the site that pulls population a next step (as strip_walk)
            const bool bot = WALLS && y == 0, top = WALLS && y == k.ny - 1;
            float id0[9], id1[9];
            id0[0] = dc.s0;                   id1[0] = dc.s1;
            id0[1] = dc.s1;                   id1[1] = dc.R;
            id0[3] = dc.L;                    id1[3] = dc.s0;
            id0[2] = top ? dc.s0 : dp.s0;     id1[2] = top ? dc.s1 : dp.s1;
            id0[5] = top ? dc.s0 : dp.s1;     id1[5] = top ? dc.s1 : dp.R;
            id0[6] = top ? dc.s0 : dp.L;      id1[6] = top ? dc.s1 : dp.s0;
            id0[4] = bot ? dc.s0 : dm.s0;     id1[4] = bot ? dc.s1 : dm.s1;
            id0[7] = bot ? dc.s0 : dm.L;      id1[7] = bot ? dc.s1 : dm.s0;
            id0[8] = bot ? dc.s0 : dm.s1;     id1[8] = bot ? dc.s1 : dm.R;
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                const float wgt = lattice_weight(a);
                st<unsigned>(out, slot_bytes<_Float16>(k, a), qb,
                             pack_f16(fmaf(f0[a], id0[a], -wgt), fmaf(f1[a], id1[a], -wgt)));
            }
            st<unsigned>(out, slot_bytes<_Float16>(k, 9), qb, pack_bf16(r0, r1));
        }
        r0 = rn0;
        r1 = rn1;
        b = a;
        db = da;
    };

    // two row buffers and two raw buffers alternate; the psi windows rotate
    float rb0 = 0.0f, rb1 = 0.0f;
    for (int i = 0; i < n; i += 2) {
        // row i: f = a, g = b; windows (pm, pc) -> pm := row y+DIR
        row(i, fa0, fa1, ra0, ra1, fb0, fb1, wb, wa, pm, pc, im, ic);
        rb0 = ra0; rb1 = ra1;
        // now pc holds row y, pm row y+DIR: swap roles so that (b, c) = (row y, row y+DIR)
        { const PairWin t = pm; pm = pc; pc = t; }
        { const PairWin t = im; im = ic; ic = t; }
        if (i + 1 >= n) break;
        row(i + 1, fb0, fb1, rb0, rb1, fa0, fa1, wa, wb, pm, pc, im, ic);
        ra0 = rb0; ra1 = rb1;
        { const PairWin t = pm; pm = pc; pc = t; }
        { const PairWin t = im; im = ic; ic = t; }
    }
    if (bad) flag[0] = kFlagUnstable;
}

// Strip `tile` of a lattice stepped with two columns per lane (k.tiles_x counts
// 124-column tiles); tiles in bands of `band` strips, as strip_tile.
template <bool WALLS, int PSI>
__device__ __forceinline__ void pair_tile(const _Float16* __restrict__ fin, _Float16* __restrict__ fout,
                                          const StepConst& k, const int tile, const int lane, int* __restrict__ flag)
{
    const int band0 = (tile / (k.tiles_x * k.band)) * k.band;
    const int band_h = min(k.band, k.tiles_y - band0);
    const int r = tile - band0 * k.tiles_x;
    const int tx = r / band_h;
    const int ty = band0 + r % band_h;
    // first column of the lane's pair; the pair index wraps in x (nx even)
    const int c0 = tx * kPairTileW - 2 + 2 * lane;
    const bool live = (lane >= 1) && (lane <= kPairTileW / 2) && (c0 < k.nx);
    const int q = c0 < 0 ? (k.nx >> 1) - 1 : (c0 >= k.nx ? 0 : (c0 >> 1));
    const unsigned qb = (unsigned)q * 4u;
    // odd strips walk towards decreasing y (as the one-column 16-bit step)
    if (ty & 1)
        pair_walk<WALLS, PSI, -1>(fin, fout, k, ty, live, qb, flag);
    else
        pair_walk<WALLS, PSI, 1>(fin, fout, k, ty, live, qb, flag);
}

template <bool WALLS, int PSI>
__global__ __launch_bounds__(kWave * kPairWaves)
__attribute__((amdgpu_waves_per_eu(1))) void d2q9_pair(
    const _Float16* __restrict__ fin, _Float16* __restrict__ fout, StepConst k, int* __restrict__ flag)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = logical_block(blockIdx.x, gridDim.x) * kPairWaves + wave;
    if (tile >= k.tiles_x * k.tiles_y) return;  // whole wavefront leaves together
    pair_tile<WALLS, PSI>(fin, fout, k, tile, lane, flag);
}

// ---------------------------------------------------------------- 24-site stencil
// Time step, moments or diagnostics with the interaction stencil of nearest and
// next-nearest neighbours (FP32 storage).  One wavefront walks a strip of 60 output
// columns (lanes 2..61; lanes 0, 1, 62, 63 are psi halo columns) and strip_rows rows,
// keeping the pulled populations of rows y, y+1, y+2 (and y+3 in flight) and the psi
// windows of rows y-2 .. y+2 in registers; x-neighbours at distance 1 and 2 come from
// lane shuffles.  Rows beyond a wall take psi of the nearest fluid row (they are
// pulled as that row).  The walk shifts its row buffers by one row per step (register
// moves), and the prefetch of row y+3 overlaps the collision of row y.
template <bool WALLS, int MODE, int PSI>
__device__ __forceinline__ void mr_walk(const float* __restrict__ fin, float* __restrict__ fout,
                                        const StepConst& k, const int tile, const int lane, const int ty,
                                        const bool live, const int xci, const unsigned xm, const unsigned xc,
                                        const unsigned xp, int* __restrict__ flag, float* __restrict__ rho_out,
                                        float* __restrict__ ux_out, float* __restrict__ uy_out, const DiagConst& dg,
                                        double* __restrict__ partial)
{
    const int y0 = ty * k.strip_rows;
    const int y1 = min(y0 + k.strip_rows, k.ny);
    const int n = y1 - y0;
    // the lattice row that supplies row y: wrapped (periodic) or clamped (walls)
    auto src = [&](int y) __attribute__((always_inline)) {
        if (WALLS) return y < 0 ? 0 : (y >= k.ny ? k.ny - 1 : y);
        return y < 0 ? y + k.ny : (y >= k.ny ? y - k.ny : y);
    };
    bool bad = false;
    // psi window of one row: columns x-2 .. x+2
    auto window = [&](float v, float (&w)[5]) __attribute__((always_inline)) {
        w[0] = __shfl_up(v, 2, kWave);
        w[1] = __shfl_up(v, 1, kWave);
        w[2] = v;
        w[3] = __shfl_down(v, 1, kWave);
        w[4] = __shfl_down(v, 2, kWave);
    };
    float f0[9], f1[9], f2[9], f3[9];
    float P[5][5];
    float r0, r1, r2;
    // rows y0-2, y0-1: psi only
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        pull_row<kStoreF32, WALLS>(fin, k, src(y0 - 2 + j), xm, xc, xp, f3);
        window(pseudopotential<PSI>(density(f3), k, bad), P[j]);
    }
    pull_row<kStoreF32, WALLS>(fin, k, src(y0), xm, xc, xp, f0);
    pull_row<kStoreF32, WALLS>(fin, k, src(y0 + 1), xm, xc, xp, f1);
    pull_row<kStoreF32, WALLS>(fin, k, src(y0 + 2), xm, xc, xp, f2);
    r0 = density(f0);
    r1 = density(f1);
    r2 = density(f2);
    window(pseudopotential<PSI>(r0, k, bad), P[2]);
    window(pseudopotential<PSI>(r1, k, bad), P[3]);
    window(pseudopotential<PSI>(r2, k, bad), P[4]);

    double acc[kDiagFields];
    if (MODE == kModeDiag) {
        for (int i = 0; i < kDiagFields; ++i) acc[i] = 0.0;
    }
    for (int i = 0; i < n; ++i) {
        const int y = y0 + i;
        // psi of row y + 3 is needed by the next row of the strip
        const bool more = i + 1 < n;
        if (more) pull_row<kStoreF32, WALLS>(fin, k, src(y + 3), xm, xc, xp, f3);
        float Fx, Fy, Fs2;
        force_stencil_mr(P, k, Fx, Fy, Fs2);
        const float jx = (f0[1] - f0[3]) + ((f0[5] - f0[7]) + (f0[8] - f0[6]));
        const float jy = (f0[2] - f0[4]) + ((f0[5] - f0[7]) + (f0[6] - f0[8]));
        const float inv_rho = recip(r0);
        const float vx = fmaf(0.5f, Fx, jx) * inv_rho;
        const float vy = fmaf(0.5f, Fy, jy) * inv_rho;
        if (MODE == kModeStep) {
            collide(f0, r0, vx, vy, Fx, Fy, Fs2, k);
            if (live) {
                float* out = fout + (long long)y * k.row_stride;
#pragma unroll
                for (int a = 0; a < 9; ++a) Codec<kStoreF32>::store(out, k, a, xc, f0[a], 0.0f);
            }
        } else if (MODE == kModeMoments) {
            if (live) write_moments(k, y, xci, r0, vx, vy, rho_out, ux_out, uy_out);
        } else {
            if (live) diag_accumulate(k, dg, y, xci, r0, vx, vy, acc);
        }
        // slide the row buffers and psi windows down by one row
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            f0[a] = f1[a];
            f1[a] = f2[a];
        }
        r0 = r1;
        r1 = r2;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int c = 0; c < 5; ++c) P[j][c] = P[j + 1][c];
        if (more) {
#pragma unroll
            for (int a = 0; a < 9; ++a) f2[a] = f3[a];
            r2 = density(f2);
            window(pseudopotential<PSI>(r2, k, bad), P[4]);
        }
    }
    if (MODE == kModeDiag) diag_write(acc, lane, tile, partial);
    if (bad) flag[0] = kFlagUnstable;
}

template <bool WALLS, int MODE, int PSI>
__global__ __launch_bounds__(kWave * kWavesPerBlock) void d2q9_mr(
    const float* __restrict__ fin, float* __restrict__ fout, StepConst k, int* __restrict__ flag,
    float* __restrict__ rho_out, float* __restrict__ ux_out, float* __restrict__ uy_out, DiagConst dg,
    double* __restrict__ partial)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = logical_block(blockIdx.x, gridDim.x) * kWavesPerBlock + wave;
    if (tile >= k.tiles_x * k.tiles_y) return;  // whole wavefront leaves together
    // tiles in bands of `band` strips, as strip_tile (k.tiles_x counts 60-column tiles)
    const int band0 = (tile / (k.tiles_x * k.band)) * k.band;
    const int band_h = min(k.band, k.tiles_y - band0);
    const int r = tile - band0 * k.tiles_x;
    const int tx = r / band_h;
    const int ty = band0 + r % band_h;
    // column of this lane; lanes 0, 1, 62, 63 are the psi halo; columns wrap in x
    const int xs = tx * kMrTileW - 2 + lane;
    const bool live = (lane >= 2) && (lane < kMrTileW + 2) && (xs < k.nx);
    int xci = xs < 0 ? xs + k.nx : (xs >= k.nx ? xs - k.nx : xs);
    if (xs > k.nx + 1) xci = 0;  // beyond the right halo: in-range dummy column, never stored
    const unsigned xc = (unsigned)xci * 4u;
    const unsigned xm = (unsigned)((xci == 0) ? k.nx - 1 : xci - 1) * 4u;
    const unsigned xp = (unsigned)((xci == k.nx - 1) ? 0 : xci + 1) * 4u;
    mr_walk<WALLS, MODE, PSI>(fin, fout, k, tile, lane, ty, live, xci, xm, xc, xp, flag, rho_out, ux_out, uy_out, dg,
                              partial);
}

// Persistent multi-instance step: one workgroup owns one lattice and advances
// it `steps` time steps; its kBatchWaves wavefronts share the strips of each step and
// meet at a workgroup barrier between steps (the barrier orders the global
// stores of step t before the loads of step t+1 for all waves of the CU).
// Workgroups never wait for each other.  Each records the wall clock at its
// start and end (for per-instance completion times).
template <int S, bool WALLS, int PSI>
__global__ __launch_bounds__(kWave * kBatchWaves) void d2q9_batch(
    const BatchInstance* __restrict__ inst, int steps, int parity,
    unsigned long long* __restrict__ clock_out)
{
    using T = typename Codec<S>::T;
    const BatchInstance& I = inst[blockIdx.x];
    const StepConst k = I.k;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ntiles = k.tiles_x * k.tiles_y;
    T* buf[2] = {reinterpret_cast<T*>(I.f[0]), reinterpret_cast<T*>(I.f[1])};
    if (threadIdx.x == 0) clock_out[2 * blockIdx.x] = wall_clock64();
    DiagConst dg{};
    for (int s = 0; s < steps; ++s) {
        const int cur = (parity + s) & 1;
        for (int tile = wave; tile < ntiles; tile += kBatchWaves)
            strip_tile<S, WALLS, kModeStep, PSI>(buf[cur], buf[cur ^ 1], k, tile, lane, I.flag, nullptr,
                                            nullptr, nullptr, dg, nullptr);
        __syncthreads();
    }
    if (threadIdx.x == 0) clock_out[2 * blockIdx.x + 1] = wall_clock64();
}

// Flat multi-instance step: one launch advances every lattice of a list by one step.
// Global tile g belongs to the lattice i with tile_start[i] <= g < tile_start[i+1];
// wg_first[b] is the lattice of workgroup b's first tile, so each wavefront
// finds its lattice by a short forward scan.  WPB wavefronts (strips) per
// workgroup, XCD-aware renumbering as the single-lattice step.
template <int WPB>
__device__ __forceinline__ const BatchInstance* flat_lattice(const BatchInstance* __restrict__ inst,
                                                             const int* __restrict__ tile_start,
                                                             const int* __restrict__ wg_first, int ntotal, int& g)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int blk = logical_block(blockIdx.x, gridDim.x);
    g = blk * WPB + wave;
    if (g >= ntotal) return nullptr;
    int i = wg_first[blk];
    while (g >= tile_start[i + 1]) ++i;
    g -= tile_start[i];
    return inst + i;
}

template <int S, bool WALLS, int PSI, int WPB>
__global__ __launch_bounds__(kWave * WPB) void d2q9_batch_flat(
    const BatchInstance* __restrict__ inst, const int* __restrict__ tile_start,
    const int* __restrict__ wg_first, int ntotal, int parity)
{
    using T = typename Codec<S>::T;
    int g;
    const BatchInstance* I = flat_lattice<WPB>(inst, tile_start, wg_first, ntotal, g);
    if (!I) return;  // whole wavefront leaves together
    const StepConst k = I->k;
    DiagConst dg{};
    strip_tile<S, WALLS, kModeStep, PSI>(reinterpret_cast<const T*>(I->f[parity]), reinterpret_cast<T*>(I->f[parity ^ 1]),
                                         k, g, threadIdx.x & (kWave - 1), I->flag, nullptr, nullptr, nullptr, dg, nullptr);
}

// The same over lattices of the destination-scaled FP16 storage with an even nx,
// stepped with two columns per lane (bitwise the one-column step).
template <bool WALLS, int PSI>
__global__ __launch_bounds__(kWave * kPairWaves) void d2q9_batch_pair(
    const BatchInstance* __restrict__ inst, const int* __restrict__ tile_start,
    const int* __restrict__ wg_first, int ntotal, int parity)
{
    int g;
    const BatchInstance* I = flat_lattice<kPairWaves>(inst, tile_start, wg_first, ntotal, g);
    if (!I) return;
    const StepConst k = I->k;
    pair_tile<WALLS, PSI>(reinterpret_cast<const _Float16*>(I->f[parity]), reinterpret_cast<_Float16*>(I->f[parity ^ 1]),
                          k, g, threadIdx.x & (kWave - 1), I->flag);
}

// Single-block, fixed-order reduction of per-wave partials (deterministic).
__global__ __launch_bounds__(256) void diag_finalize(const double* __restrict__ partial, int ntiles,
                                                     double* __restrict__ out)
{
    __shared__ double sh[256][kDiagFields];
    double acc[kDiagFields];
    for (int i = 0; i < kDiagFields; ++i) acc[i] = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += 256) {
        for (int i = 0; i < 9; ++i) acc[i] += partial[(long long)t * kDiagFields + i];
        acc[9] = fmax(acc[9], partial[(long long)t * kDiagFields + 9]);
    }
    for (int i = 0; i < kDiagFields; ++i) sh[threadIdx.x][i] = acc[i];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int i = 0; i < 9; ++i) sh[threadIdx.x][i] += sh[threadIdx.x + s][i];
            sh[threadIdx.x][9] = fmax(sh[threadIdx.x][9], sh[threadIdx.x + s][9]);
        }
        __syncthreads();
    }
    if (threadIdx.x < kDiagFields) out[threadIdx.x] = sh[0][threadIdx.x];
}

// Initial state.  Slot (z, b) of the stored (pre-streamed) buffer holds the
// value the first pull will read: f_eq_b at z + e_b, or, where z + e_b lies
// beyond a wall, f_eq_bbar at z (it comes back by bounce-back).
// f_eq = M^-1 m_eq(rho, u) of Eq. (3), i.e. w_a rho (1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u^2),
// evaluated in FP64 and rounded once, so that the stored values sum to rho0 to
// within the rounding of each population.
template <int S, bool WALLS, int REACH>
__global__ __launch_bounds__(256) void d2q9_init(const float* __restrict__ rho0,
                                                 const float* __restrict__ ux0,
                                                 const float* __restrict__ uy0,
                                                 typename Codec<S>::T* __restrict__ fout,
                                                 StepConst k, InitConst ic, int* __restrict__ flag)
{
    using C = Codec<S>;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= k.nx) return;
    constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    constexpr double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    {
        // validate this site's input
        const long long i = (long long)y * k.nx + x;
        const float r = rho0[i];
        const float ux = ux0 ? ux0[i] : 0.0f, uy = uy0 ? uy0[i] : 0.0f;
        bool bad = !(r > 0.0f) || !isfinite(ux) || !isfinite(uy) || !isfinite(r);
        if (!bad) {
            if (ic.psi.form == kPsiSS) pseudopotential<kPsiSS>(r, k, bad);
            else pseudopotential<kPsiCS>(r, k, bad);
        }
        if (bad) flag[0] = kFlagBadInput;
    }
    // psi (FP64, Eq. (24) or Eq. (23)) on the block of half-width REACH + 1 around
    // (x, y): the force of Eq. (7) at the nine sites this one pulls from, for a stencil
    // of reach REACH.  Rows beyond a wall take the nearest fluid row; they are read only
    // by sites inside the lattice.
    constexpr int HB = REACH + 1, NB = 2 * HB + 1;
    double psi[NB][NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        int yy = y + j - HB;
        if (WALLS) yy = yy < 0 ? 0 : (yy >= k.ny ? k.ny - 1 : yy);
        else yy = ((yy % k.ny) + k.ny) % k.ny;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int xx = ((x + i - HB) % k.nx + k.nx) % k.nx;
            const double r = rho0[(long long)yy * k.nx + xx];
            psi[j][i] = sqrt(psi2_f64(r, ic.psi));
        }
    }
    // (the nine upstream forces are unrolled for the nearest-neighbour stencil only: the
    // 24-site stencil's fully unrolled block is large enough to crash the instruction
    // scheduler, and this kernel runs once per lattice)
    constexpr int kUnrollForces = REACH == 1 ? 9 : 1;
#pragma unroll kUnrollForces
    for (int b = 0; b < 9; ++b) {
        // pre-streamed: slot b of (x, y) holds what the first pull of direction b
        // reads, the equilibrium of the upstream site (or of this site's
        // opposite direction at a wall)
        int dx = EX[b], dy = EY[b];
        int a = b;
        int ys = y + dy;
        if (ys < 0 || ys >= k.ny) {
            if (WALLS) { dx = 0; dy = 0; a = OPP[b]; }
            else ys = ys < 0 ? ys + k.ny : ys - k.ny;
        }
        if (WALLS) ys = y + dy;
        int xs = x + dx;
        xs = xs < 0 ? xs + k.nx : (xs >= k.nx ? xs - k.nx : xs);
        // Eq. (7) at the upstream site: the nearest-neighbour weights 1/3, 1/12, or the
        // 24-site weights 4/21, 4/45, 1/60, 2/315, 1/5040 by |e|^2 = 1, 2, 4, 5, 8
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int ey = -REACH; ey <= REACH; ++ey)
#pragma unroll
            for (int ex = -REACH; ex <= REACH; ++ex) {
                const int q = ex * ex + ey * ey;
                double w = 0.0;
                if (REACH == 1) w = q == 1 ? 1.0 / 3.0 : (q == 2 ? 1.0 / 12.0 : 0.0);
                else w = q == 1 ? 4.0 / 21.0 : q == 2 ? 4.0 / 45.0 : q == 4 ? 1.0 / 60.0 : q == 5 ? 2.0 / 315.0
                       : q == 8 ? 1.0 / 5040.0 : 0.0;
                const double ps = psi[HB + dy + ey][HB + dx + ex];
                sx += w * ps * ex;
                sy += w * ps * ey;
            }
        const double pc = psi[HB + dy][HB + dx];
        const double Fx = -ic.psi.G * pc * sx, Fy = -ic.psi.G * pc * sy;
        const long long i = (long long)ys * k.nx + xs;
        const double r = rho0[i];
        // Eq. (6): the equilibrium velocity is u0 - F / (2 rho0), so that the
        // moments at t = 0 return u0
        const double ux = (ux0 ? ux0[i] : 0.0) - Fx / (2.0 * r);
        const double uy = (uy0 ? uy0[i] : 0.0) - Fy / (2.0 * r);
        const double eu = EX[a] * ux + EY[a] * uy;
        const double feq = W[a] * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy));
        C::store_init(fout + (long long)y * k.row_stride, k, b, (unsigned)x * (unsigned)sizeof(typename C::T),
                      feq, (double)rho0[(long long)y * k.nx + x], r);
    }
}

// One 16-byte element per thread: the fastest plain copy form on gfx950.
__global__ __launch_bounds__(256) void copy_probe(const float4* __restrict__ src,
                                                  float4* __restrict__ dst, long long n)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ---------------------------------------------------------------- launchers

// Dynamic LDS that caps the resident workgroups of a strip kernel at `cap` per CU
// (0: no cap).  The one-column destination-scaled FP16 step runs fastest with five 4-wave
// workgroups per CU (measured on the 8192 x 4096 splash: 107.9k MLUPS, against
// 102.8k with the six its registers allow and 105.5k with four); the LDS is
// reserved only to limit occupancy and is never accessed.
static size_t occupancy_cap_lds(int cap)
{
    static size_t per_cu = 0;
    if (cap <= 0) return 0;
    if (per_cu == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
            v <= 0)
            return 0;
        per_cu = (size_t)v;
    }
    // more than per_cu / (cap + 1) bytes each: at most `cap` workgroups fit
    return per_cu / (size_t)(cap + 1) + 256;
}

constexpr int kDestBlocksPerCu = 5;  // one-column destination-scaled FP16 step (see occupancy_cap_lds)

static int strip_blocks(const StepConst& k, int waves_per_block)
{
    const long long tiles = (long long)k.tiles_x * k.tiles_y;
    return (int)((tiles + waves_per_block - 1) / waves_per_block);
}

template <int S, bool WALLS, int MODE, int PSI>
static hipError_t launch_mode(const void* fin, void* fout, const StepConst& k, int* flag,
                              float* rho, float* ux, float* uy, const DiagConst& dg,
                              double* partial, hipStream_t s)
{
    using T = typename Codec<S>::T;
    constexpr int wpb = step_waves_per_block(S);
    const size_t lds = occupancy_cap_lds(S == kStoreF16Dest ? kDestBlocksPerCu : 0);
    hipLaunchKernelGGL((d2q9_strip<S, WALLS, MODE, PSI>), dim3(strip_blocks(k, wpb)),
                       dim3(kWave * wpb), lds, s, static_cast<const T*>(fin),
                       static_cast<T*>(fout), k, flag, rho, ux, uy, dg, partial);
    return hipGetLastError();
}

// the pseudopotential form of k selects the instantiation
template <int MODE, int S, bool WALLS>
static hipError_t launch_psi(const void* fin, void* fout, const StepConst& k, int* flag,
                             float* rho, float* ux, float* uy, const DiagConst& dg,
                             double* partial, hipStream_t s)
{
    return k.psi_form == kPsiSS
               ? launch_mode<S, WALLS, MODE, kPsiSS>(fin, fout, k, flag, rho, ux, uy, dg, partial, s)
               : launch_mode<S, WALLS, MODE, kPsiCS>(fin, fout, k, flag, rho, ux, uy, dg, partial, s);
}

template <int MODE>
static hipError_t dispatch(int store, bool walls, const void* fin, void* fout, const StepConst& k,
                           int* flag, float* rho, float* ux, float* uy, const DiagConst& dg,
                           double* partial, hipStream_t s)
{
    switch (store) {
    case kStoreF32:
        return walls ? launch_psi<MODE, kStoreF32, true>(fin, fout, k, flag, rho, ux, uy, dg, partial, s)
                     : launch_psi<MODE, kStoreF32, false>(fin, fout, k, flag, rho, ux, uy, dg, partial, s);
    case kStoreF16:
        return walls ? launch_psi<MODE, kStoreF16, true>(fin, fout, k, flag, rho, ux, uy, dg, partial, s)
                     : launch_psi<MODE, kStoreF16, false>(fin, fout, k, flag, rho, ux, uy, dg, partial, s);
    case kStoreBF16:
        return walls ? launch_psi<MODE, kStoreBF16, true>(fin, fout, k, flag, rho, ux, uy, dg, partial, s)
                     : launch_psi<MODE, kStoreBF16, false>(fin, fout, k, flag, rho, ux, uy, dg, partial, s);
    case kStoreF16Local:
        return walls ? launch_psi<MODE, kStoreF16Local, true>(fin, fout, k, flag, rho, ux, uy, dg, partial, s)
                     : launch_psi<MODE, kStoreF16Local, false>(fin, fout, k, flag, rho, ux, uy, dg, partial, s);
    case kStoreBF16Local:
        return walls ? launch_psi<MODE, kStoreBF16Local, true>(fin, fout, k, flag, rho, ux, uy, dg, partial, s)
                     : launch_psi<MODE, kStoreBF16Local, false>(fin, fout, k, flag, rho, ux, uy, dg, partial, s);
    case kStoreF16Dest:
        return walls ? launch_psi<MODE, kStoreF16Dest, true>(fin, fout, k, flag, rho, ux, uy, dg, partial, s)
                     : launch_psi<MODE, kStoreF16Dest, false>(fin, fout, k, flag, rho, ux, uy, dg, partial, s);
    default:
        return hipErrorInvalidValue;
    }
}

int step_blocks_per_cu(int store, bool walls)
{
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
#define LBMP_OCC(S_, W_)                                                                              \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, d2q9_strip<S_, W_, kModeStep, kPsiCS>,              \
                                                     kWave * step_waves_per_block(S_), 0)
    switch (store) {
    case kStoreF32: if (walls) LBMP_OCC(kStoreF32, true); else LBMP_OCC(kStoreF32, false); break;
    case kStoreF16: if (walls) LBMP_OCC(kStoreF16, true); else LBMP_OCC(kStoreF16, false); break;
    case kStoreBF16: if (walls) LBMP_OCC(kStoreBF16, true); else LBMP_OCC(kStoreBF16, false); break;
    case kStoreF16Local: if (walls) LBMP_OCC(kStoreF16Local, true); else LBMP_OCC(kStoreF16Local, false); break;
    case kStoreBF16Local: if (walls) LBMP_OCC(kStoreBF16Local, true); else LBMP_OCC(kStoreBF16Local, false); break;
    case kStoreF16Dest: if (walls) LBMP_OCC(kStoreF16Dest, true); else LBMP_OCC(kStoreF16Dest, false); break;
    default: break;
    }
#undef LBMP_OCC
    return e == hipSuccess ? nb : 0;
}

// The two-columns-per-lane step of the destination-scaled FP16 storage (even nx).
template <bool WALLS, int PSI>
static hipError_t launch_pair_psi(const void* fin, void* fout, const StepConst& k, int* flag, hipStream_t s)
{
    StepConst kp = k;
    kp.tiles_x = (k.nx + kPairTileW - 1) / kPairTileW;
    const long long tiles = (long long)kp.tiles_x * kp.tiles_y;
    const int blocks = (int)((tiles + kPairWaves - 1) / kPairWaves);
    hipLaunchKernelGGL((d2q9_pair<WALLS, PSI>), dim3(blocks), dim3(kWave * kPairWaves),
                       0, s, static_cast<const _Float16*>(fin),
                       static_cast<_Float16*>(fout), kp, flag);
    return hipGetLastError();
}

bool pair_step(int store, int nx)
{
    return store == kStoreF16Dest && nx % 2 == 0 && nx >= 4;
}

int pair_blocks_per_cu(bool walls)
{
    int nb = 0;
    const hipError_t e =
        walls ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, d2q9_pair<true, kPsiCS>, kWave * kPairWaves, 0)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, d2q9_pair<false, kPsiCS>, kWave * kPairWaves, 0);
    return e == hipSuccess ? nb : 0;
}

// The 24-site stencil (FP32 storage; the host validates that): step, moments or
// diagnostics by MODE.  k.tiles_x counts 60-column tiles.
template <int MODE>
static hipError_t launch_mr(bool walls, const void* fin, void* fout, const StepConst& k, int* flag, float* rho,
                            float* ux, float* uy, const DiagConst& dg, double* partial, hipStream_t s)
{
    const dim3 grid(strip_blocks(k, kWavesPerBlock)), block(kWave * kWavesPerBlock);
    const float* in = static_cast<const float*>(fin);
    float* out = static_cast<float*>(fout);
#define LBMP_MR(W_, P_)                                                                            \
    hipLaunchKernelGGL((d2q9_mr<W_, MODE, P_>), grid, block, 0, s, in, out, k, flag, rho, ux, uy, dg, partial)
    if (walls) {
        if (k.psi_form == kPsiSS) LBMP_MR(true, kPsiSS); else LBMP_MR(true, kPsiCS);
    } else {
        if (k.psi_form == kPsiSS) LBMP_MR(false, kPsiSS); else LBMP_MR(false, kPsiCS);
    }
#undef LBMP_MR
    return hipGetLastError();
}

hipError_t launch_step(int store, bool walls, const void* fin, void* fout, const StepConst& k,
                       int* flag, hipStream_t s)
{
    if (k.stencil == kStencilMultirange) {
        if (store != kStoreF32) return hipErrorInvalidValue;
        return launch_mr<kModeStep>(walls, fin, fout, k, flag, nullptr, nullptr, nullptr, DiagConst{}, nullptr, s);
    }
    if (pair_step(store, k.nx)) {
        if (walls)
            return k.psi_form == kPsiSS ? launch_pair_psi<true, kPsiSS>(fin, fout, k, flag, s)
                                        : launch_pair_psi<true, kPsiCS>(fin, fout, k, flag, s);
        return k.psi_form == kPsiSS ? launch_pair_psi<false, kPsiSS>(fin, fout, k, flag, s)
                                    : launch_pair_psi<false, kPsiCS>(fin, fout, k, flag, s);
    }
    DiagConst dg{};
    return dispatch<kModeStep>(store, walls, fin, fout, k, flag, nullptr, nullptr, nullptr, dg,
                               nullptr, s);
}

hipError_t launch_batch(int store, bool walls, int psi, const BatchInstance* inst, int n, int steps,
                        int parity, unsigned long long* clocks, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
#define LBMP_BATCH(S_, W_)                                                                         \
    do {                                                                                           \
        if (psi == kPsiSS)                                                                         \
            hipLaunchKernelGGL((d2q9_batch<S_, W_, kPsiSS>), dim3(n), dim3(kWave * kBatchWaves), 0, s, \
                               inst, steps, parity, clocks);                                       \
        else                                                                                       \
            hipLaunchKernelGGL((d2q9_batch<S_, W_, kPsiCS>), dim3(n), dim3(kWave * kBatchWaves), 0, s, \
                               inst, steps, parity, clocks);                                       \
    } while (0)
    switch (store) {
    case kStoreF32: if (walls) LBMP_BATCH(kStoreF32, true); else LBMP_BATCH(kStoreF32, false); break;
    case kStoreF16Local: if (walls) LBMP_BATCH(kStoreF16Local, true); else LBMP_BATCH(kStoreF16Local, false); break;
    case kStoreF16Dest: if (walls) LBMP_BATCH(kStoreF16Dest, true); else LBMP_BATCH(kStoreF16Dest, false); break;
    default: return hipErrorInvalidValue;
    }
#undef LBMP_BATCH
    return hipGetLastError();
}

int batch_waves_per_block(int store, bool pair)
{
    if (pair) return kPairWaves;
    return store == kStoreF16Dest ? kBatchWavesDest : kWavesPerBlock;
}

hipError_t launch_batch_flat(int store, bool walls, int psi, bool pair, const BatchInstance* inst,
                             const int* tile_start, const int* wg_first, int ntotal, int parity, hipStream_t s)
{
    if (ntotal <= 0) return hipSuccess;
    const int wpb = batch_waves_per_block(store, pair);
    const int blocks = (ntotal + wpb - 1) / wpb;
    if (pair) {
        if (store != kStoreF16Dest) return hipErrorInvalidValue;
#define LBMP_PAIRB(W_, P_)                                                                         \
    hipLaunchKernelGGL((d2q9_batch_pair<W_, P_>), dim3(blocks), dim3(kWave * kPairWaves), 0, s, inst, \
                       tile_start, wg_first, ntotal, parity)
        if (walls) {
            if (psi == kPsiSS) LBMP_PAIRB(true, kPsiSS); else LBMP_PAIRB(true, kPsiCS);
        } else {
            if (psi == kPsiSS) LBMP_PAIRB(false, kPsiSS); else LBMP_PAIRB(false, kPsiCS);
        }
#undef LBMP_PAIRB
        return hipGetLastError();
    }
#define LBMP_FLAT(S_, W_, N_)                                                                      \
    do {                                                                                           \
        if (psi == kPsiSS)                                                                         \
            hipLaunchKernelGGL((d2q9_batch_flat<S_, W_, kPsiSS, N_>), dim3(blocks), dim3(kWave * N_), \
                               0, s, inst, tile_start, wg_first, ntotal, parity);                  \
        else                                                                                       \
            hipLaunchKernelGGL((d2q9_batch_flat<S_, W_, kPsiCS, N_>), dim3(blocks), dim3(kWave * N_), \
                               0, s, inst, tile_start, wg_first, ntotal, parity);                  \
    } while (0)
    switch (store) {
    case kStoreF32: if (walls) LBMP_FLAT(kStoreF32, true, kWavesPerBlock); else LBMP_FLAT(kStoreF32, false, kWavesPerBlock); break;
    case kStoreF16Local: if (walls) LBMP_FLAT(kStoreF16Local, true, kWavesPerBlock); else LBMP_FLAT(kStoreF16Local, false, kWavesPerBlock); break;
    case kStoreF16Dest: if (walls) LBMP_FLAT(kStoreF16Dest, true, kBatchWavesDest); else LBMP_FLAT(kStoreF16Dest, false, kBatchWavesDest); break;
    default: return hipErrorInvalidValue;
    }
#undef LBMP_FLAT
    return hipGetLastError();
}

hipError_t launch_moments(int store, bool walls, const void* fin, const StepConst& k, int* flag,
                          float* rho, float* ux, float* uy, hipStream_t s)
{
    DiagConst dg{};
    if (k.stencil == kStencilMultirange) {
        if (store != kStoreF32) return hipErrorInvalidValue;
        return launch_mr<kModeMoments>(walls, fin, nullptr, k, flag, rho, ux, uy, dg, nullptr, s);
    }
    return dispatch<kModeMoments>(store, walls, fin, nullptr, k, flag, rho, ux, uy, dg, nullptr, s);
}

hipError_t launch_diag(int store, bool walls, const void* fin, const StepConst& k, int* flag,
                       const DiagConst& dg, double* partial, double* out, hipStream_t s)
{
    hipError_t e = hipSuccess;
    if (k.stencil == kStencilMultirange)
        e = store == kStoreF32 ? launch_mr<kModeDiag>(walls, fin, nullptr, k, flag, nullptr, nullptr, nullptr, dg,
                                                      partial, s)
                               : hipErrorInvalidValue;
    else
        e = dispatch<kModeDiag>(store, walls, fin, nullptr, k, flag, nullptr, nullptr, nullptr, dg, partial, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(diag_finalize, dim3(1), dim3(256), 0, s, partial, k.tiles_x * k.tiles_y, out);
    return hipGetLastError();
}

hipError_t launch_init(int store, bool walls, const float* rho0, const float* ux0,
                       const float* uy0, void* fout, const StepConst& k, const InitConst& ic, int* flag,
                       hipStream_t s)
{
    dim3 grid((k.nx + 255) / 256, k.ny), block(256);
#define LBMP_INIT(S_, W_)                                                                          \
    do {                                                                                           \
        if (k.stencil == kStencilMultirange)                                                       \
            hipLaunchKernelGGL((d2q9_init<S_, W_, 2>), grid, block, 0, s, rho0, ux0, uy0,          \
                               static_cast<typename Codec<S_>::T*>(fout), k, ic, flag);            \
        else                                                                                       \
            hipLaunchKernelGGL((d2q9_init<S_, W_, 1>), grid, block, 0, s, rho0, ux0, uy0,          \
                               static_cast<typename Codec<S_>::T*>(fout), k, ic, flag);            \
    } while (0)
    switch (store) {
    case kStoreF32: if (walls) LBMP_INIT(kStoreF32, true); else LBMP_INIT(kStoreF32, false); break;
    case kStoreF16: if (walls) LBMP_INIT(kStoreF16, true); else LBMP_INIT(kStoreF16, false); break;
    case kStoreBF16: if (walls) LBMP_INIT(kStoreBF16, true); else LBMP_INIT(kStoreBF16, false); break;
    case kStoreF16Local: if (walls) LBMP_INIT(kStoreF16Local, true); else LBMP_INIT(kStoreF16Local, false); break;
    case kStoreBF16Local: if (walls) LBMP_INIT(kStoreBF16Local, true); else LBMP_INIT(kStoreBF16Local, false); break;
    case kStoreF16Dest: if (walls) LBMP_INIT(kStoreF16Dest, true); else LBMP_INIT(kStoreF16Dest, false); break;
    default: return hipErrorInvalidValue;
    }
#undef LBMP_INIT
    return hipGetLastError();
}

hipError_t launch_copy_probe(const void* src, void* dst, long long n16, hipStream_t s)
{
    const long long blocks = (n16 + 255) / 256;
    if (blocks < 1 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(copy_probe, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const float4*>(src), static_cast<float4*>(dst), n16);
    return hipGetLastError();
}

}  // namespace lbmp
