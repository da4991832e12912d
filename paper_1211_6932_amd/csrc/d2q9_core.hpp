// d2q9_core.hpp -- device code of the improved MRT pseudopotential D2Q9 step
// (Li, Luo & Li, arXiv:1211.6932) for gfx950.
//
// Layout in HBM: the stored state is the post-collision distribution f*
// (pull streaming), row-interleaved structure of arrays f[y][alpha][pitch]: the
// nine population rows of one lattice row are contiguous, x fastest, and the
// rows are packed without padding (pitch = nx, rounded to even for the
// local-density encodings), so the whole state is one contiguous stream.  A
// row's pull then reads three contiguous blocks (rows y-1, y, y+1) and its store
// writes one, instead of touching 18 separate planes.  Two such buffers
// ping-pong.
//
// Work decomposition: one 64-lane wavefront owns a strip of 62 output columns
// and `strip_rows` rows.  Lane l handles column x0 - 1 + l; lanes 0 and 63 are
// halo columns that only evaluate the pseudopotential psi.  The wave walks
// down the strip keeping psi of rows y-1, y, y+1 in registers; the x-neighbours
// of psi come from the adjacent lanes by cross-lane shuffles, so the stencil of
// Eq. (7) needs neither LDS nor workgroup barriers.  Rows y0-1 and y1 are
// pulled once more per strip to provide the y-halo of psi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmp {

constexpr int kWave = 64;
constexpr int kTileW = kWave - 2;     // output columns per wavefront strip
constexpr int kPairTileW = 2 * kWave - 4;  // output columns per wavefront, two columns per lane
constexpr int kMrTileW = kWave - 4;   // output columns per wavefront, 24-site stencil (two halo lanes a side)
constexpr int kPairWaves = 4;         // wavefronts per workgroup, two columns per lane
constexpr int kWavesPerBlock = 16;    // wavefronts (strips) per workgroup: FP32 step, FP32 batch
constexpr int kBatchWaves = 16;       // wavefronts per workgroup (= per lattice) of the persistent batch
// Wavefronts per workgroup of the flat batch with destination-scaled FP16, one column
// per lane (FP32 and source-density FP16 use kWavesPerBlock).  On the 512-lattice
// sweep: 100.7k MLUPS with 4 against 98.7k with 16 (source-density FP16: 78.9k with 4,
// 80.1k with 16).
constexpr int kBatchWavesDest = 4;
constexpr int kNumXcd = 8;            // MI355X: 8 accelerator complex dies, one L2 each
constexpr int kDiagFields = 10;       // doubles per wave partial in the diagnostics pass

enum : int { kStoreF32 = 0, kStoreF16 = 1, kStoreBF16 = 2, kStoreF16Local = 3, kStoreBF16Local = 4, kStoreF16Dest = 5 };

// Wavefronts per workgroup of the single-lattice strip kernels, by storage.  The
// FP32 step is bound by HBM and streams best with one 16-wave workgroup per CU
// (the resident waves then cover the fewest rows); the destination-scaled FP16
// step is bound by latency and issue, and gains from more, smaller workgroups
// per CU (measured on the 8192 x 4096 splash: 106k vs 98k MLUPS with 4 waves).
constexpr int step_waves_per_block(int store)
{
    return store == kStoreF16Dest ? 4 : kWavesPerBlock;
}
enum : int { kModeStep = 0, kModeMoments = 1, kModeDiag = 2 };
enum : int { kFlagUnstable = 1, kFlagBadInput = 2 };
enum : int { kPsiCS = 0, kPsiSS = 1 };  // psi of Eq. (24) from Eq. (30), or of Eq. (23)
enum : int { kStencilNearest = 0, kStencilMultirange = 1 };  // interaction stencil of Eq. (7)

// Per-launch constants (FP32 copies of FP64 host-derived values).
struct StepConst {
    int nx, ny, pitch;          // pitch in elements
    int tiles_x, tiles_y, strip_rows;
    int band;                   // strips per tile band: consecutive tiles walk down `band` strips, then right
    long long row_stride;       // elements of the storage type per lattice row (9 or 11 pitches)
    float b4;                   // b / 4
    float RT;                   // R T
    float a;                    // attraction constant of Eq. (30)
    float two_over_G;           // 2 / G  (Eq. 24 with c = 1)
    float negG;                 // -G     (Eq. 7)
    float rho_switch;           // nu_l for rho >= rho_switch, nu_g below
    // Relaxation of the non-conserved moments (Eqs. 2-4, 25), with the column norms of
    // M^-1 folded in (e, eps: 36; q: 12; p: 4): for the e moment
    //   (m*_e - m_e) / 36 = -a_e (m_e - m_e^eq) + b_e v.F + c_e |Fs|^2,
    // a_e = s_e / 36, b_e = 6 (1 - s_e/2) / 36, c_e = 12 sigma G^2 s_e / 36, and
    // likewise for eps (a_z, b_z, c_z), q (a_q = s_q / 12, b_q = (1 - s_q/2) / 12) and
    // the two shear moments (a_nu = s_nu / 4 per phase; b_nu = (1 - s_nu/2) / 2 for
    // p_xx, whose forcing term is 2 (vx Fx - vy Fy), and half of it for p_xy).
    float a_e, b_e, c_e, a_z, b_z, c_z, a_q, b_q;
    float a_nu_l, b_nu_l, a_nu_g, b_nu_g;
    int psi_form;               // kPsiCS or kPsiSS
    int stencil;                // kStencilNearest or kStencilMultirange
    float psi_eps, inv_psi_eps; // epsilon of Eq. (23) and 1/epsilon (0 when epsilon = 0)
    float off[9];               // w_a rho_ref: offsets of the 16-bit storage (0 for FP32)
};

// One lattice of a batched launch: its constants, its two state buffers and
// its unstable flag.
struct BatchInstance {
    StepConst k;
    void* f[2];
    int* flag;
};

// Diagnostics regions (annuli) and output.
// FP64 parameters of the pseudopotential: Eq. (24) with Eq. (30), or Eq. (23).
struct PsiConst {
    double b4, RT, a, G;
    double eps;     // epsilon of Eq. (23)
    int form;       // kPsiCS or kPsiSS
};

// FP64 parameters of the initial-state kernel (Eqs. (7), (23)/(24), (30)).
struct InitConst {
    PsiConst psi;
};

struct DiagConst {
    double in_cx, in_cy, in_r0, in_r1;
    double out_cx, out_cy, out_r0, out_r1;
    PsiConst psi;  // FP64 copies for the bulk pressure
    int periodic_y;
};

// ---------------------------------------------------------------- storage codecs
// Element access by 32-bit byte offset from a (wave-uniform) row pointer (the
// initial-state kernel).  Valid because a lattice row is limited to < 4 GiB
// (host validation).
template <class T>
__device__ __forceinline__ T& at(T* p, unsigned byte_off)
{
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(p) + byte_off);
}
template <class T>
__device__ __forceinline__ const T& at(const T* p, unsigned byte_off)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + byte_off);
}

// Step-loop accesses go through buffer instructions: a buffer resource made from
// the (wave-uniform) start of a lattice row, the population slot's byte offset
// as the scalar offset and the column's byte offset as the 32-bit vector offset.
// The hardware adds the three, so no 64-bit address is formed per lane and
// access, and the nine slots of a row share one resource.  The record count is
// the maximum, so no range check applies (every offset stays inside the row,
// which host validation keeps below 4 GiB).
constexpr int kRsrcFlags = 0x00020000;  // dword 3 of a raw (stride 0) gfx9 buffer resource

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* row)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(row), (short)0, (int)0xffffffff, kRsrcFlags);
}

// The slot offset is wave-uniform by construction; saying so keeps it in a
// scalar register (a value the compiler cannot prove uniform would otherwise be
// served by a loop over its distinct lane values).
__device__ __forceinline__ int uniform(unsigned v) { return __builtin_amdgcn_readfirstlane((int)v); }

template <class T>
__device__ __forceinline__ T ld(const void* row, unsigned slot_off, unsigned col)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 2, "32- or 16-bit elements");
    const __amdgpu_buffer_rsrc_t r = row_rsrc(row);
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)col, uniform(slot_off), 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, (int)col, uniform(slot_off), 0));
}
template <class T>
__device__ __forceinline__ void st(void* row, unsigned slot_off, unsigned col, T v)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 2, "32- or 16-bit elements");
    const __amdgpu_buffer_rsrc_t r = row_rsrc(row);
    if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)col, uniform(slot_off), 0);
    else
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)col, uniform(slot_off), 0);
}

// Byte offset of population slot a (or the density slots, a = 9) within a lattice row.
template <class T>
__device__ __forceinline__ unsigned slot_bytes(const StepConst& k, int a)
{
    return (unsigned)a * (unsigned)k.pitch * (unsigned)sizeof(T);
}

// Lattice weight of population a (4/9 rest, 1/9 axis, 1/36 diagonal).
__device__ __forceinline__ float lattice_weight(int a)
{
    return a == 0 ? 4.0f / 9.0f : (a < 5 ? 1.0f / 9.0f : 1.0f / 36.0f);
}

// Codecs address one lattice row: `row` points at its start, `a` is the stored
// population read or written, `col` the byte offset of the column for
// elements of type T.  The nine population rows of a lattice row are `pitch`
// elements apart.  store() receives 1/rho of the site (used by the
// local-density encodings only).
template <int S> struct Codec;

template <> struct Codec<kStoreF32> {
    using T = float;
    static constexpr int kRowSlots = 9;  // T-sized row slots per lattice row
    static constexpr bool kDestScaled = false;
    static __device__ __forceinline__ float load(const T* row, const StepConst& k, int a, unsigned col) {
        return ld<T>(row, slot_bytes<T>(k, a), col);
    }
    static __device__ __forceinline__ void store(T* row, const StepConst& k, int a, unsigned col, float v, float) {
        st<T>(row, slot_bytes<T>(k, a), col, v);
    }
    static __device__ __forceinline__ void store_density(T*, const StepConst&, unsigned, float) {}
    static __device__ __forceinline__ void store_init(T* row, const StepConst& k, int a, unsigned col, double v, double,
                                                      double) {
        at(row + a * k.pitch, col) = static_cast<float>(v);
    }
};

// 16-bit offsets from the rest equilibrium of one fixed reference density:
// stored h_a = f_a - w_a rho_ref (k.off[a] = w_a rho_ref).
template <class H> struct CodecGlobal {
    using T = H;
    static constexpr int kRowSlots = 9;
    static constexpr bool kDestScaled = false;
    static __device__ __forceinline__ float load(const T* row, const StepConst& k, int a, unsigned col) {
        return static_cast<float>(ld<T>(row, slot_bytes<T>(k, a), col)) + k.off[a];
    }
    static __device__ __forceinline__ void store(T* row, const StepConst& k, int a, unsigned col, float v, float) {
        st<T>(row, slot_bytes<T>(k, a), col, static_cast<T>(v - k.off[a]));  // round to nearest even
    }
    static __device__ __forceinline__ void store_density(T*, const StepConst&, unsigned, float) {}
    static __device__ __forceinline__ void store_init(T* row, const StepConst& k, int a, unsigned col, double v, double,
                                                      double) {
        at(row + a * k.pitch, col) = static_cast<T>(static_cast<float>(v - (double)k.off[a]));
    }
};

// 16-bit relative offsets from the rest equilibrium of the site's own
// density: each lattice row stores g_a = f*_a / rho - w_a (nine 16-bit rows)
// followed by rho in FP32 (two 16-bit slots per column), so f*_a = rho (w_a + g_a).
// A pulled value is decoded with the density of the site it was streamed from.
// Relative offsets keep the vapour values (rho ~ 1e-4) in the normal range of
// FP16, where an absolute offset would fall into its subnormals.
template <class H> struct CodecLocal {
    using T = H;
    static constexpr int kRowSlots = 11;
    static constexpr bool kDestScaled = false;
    static __device__ __forceinline__ float load(const T* row, const StepConst& k, int a, unsigned col) {
        const float rho = ld<float>(row, slot_bytes<T>(k, 9), 2u * col);
        return rho * (lattice_weight(a) + static_cast<float>(ld<T>(row, slot_bytes<T>(k, a), col)));
    }
    static __device__ __forceinline__ void store(T* row, const StepConst& k, int a, unsigned col, float v,
                                                 float inv_rho) {
        st<T>(row, slot_bytes<T>(k, a), col, static_cast<T>(fmaf(v, inv_rho, -lattice_weight(a))));
    }
    static __device__ __forceinline__ void store_density(T* row, const StepConst& k, unsigned col, float rho) {
        st<float>(row, slot_bytes<T>(k, 9), 2u * col, rho);
    }
    static __device__ __forceinline__ void store_init(T* row, const StepConst& k, int a, unsigned col, double v,
                                                      double rho, double) {
        const double w = a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        const float r = static_cast<float>(rho);
        at(row + a * k.pitch, col) = static_cast<T>(static_cast<float>(v / (double)r - w));
        if (a == 0) at(reinterpret_cast<float*>(row + 9 * k.pitch), 2u * col) = r;
    }
};

// 16-bit relative offsets scaled by the density of the site that will pull the
// value: slot a of site s holds g_a = f*_a(s) / rhohat(d) - w_a, d = s + e_a
// (d = s for a population that reflects at a wall), and each site stores
// rhohat = bf16(rho) of its own density once.  The puller d then decodes all
// nine populations with its own rhohat: f_a = rhohat(d) (w_a + g_a), one
// density load per site instead of nine.  The encoder takes rhohat of the
// eight neighbours from the density window it keeps for the force stencil;
// every lane computing a site's density gets the same bits, so encoder and
// decoder use the same scale.  The scale only needs to be consistent, not
// precise: its bf16 rounding is absorbed in g.
struct CodecDest {
    using T = _Float16;
    static constexpr int kRowSlots = 10;
    static constexpr bool kDestScaled = true;
    static __device__ __forceinline__ float round_scale(float rho) {
        return static_cast<float>(static_cast<__bf16>(rho));
    }
    static __device__ __forceinline__ float scale(const T* row, const StepConst& k, unsigned col) {
        return static_cast<float>(ld<__bf16>(row, slot_bytes<T>(k, 9), col));
    }
    // g_a only: pull_row forms rhohat g_a + rhohat w_a with the puller's own scale
    static __device__ __forceinline__ float load(const T* row, const StepConst& k, int a, unsigned col) {
        return static_cast<float>(ld<T>(row, slot_bytes<T>(k, a), col));
    }
    static __device__ __forceinline__ void store(T* row, const StepConst& k, int a, unsigned col, float v,
                                                 float inv_scale_dest) {
        st<T>(row, slot_bytes<T>(k, a), col, static_cast<T>(fmaf(v, inv_scale_dest, -lattice_weight(a))));
    }
    static __device__ __forceinline__ void store_density(T* row, const StepConst& k, unsigned col, float rho) {
        st<__bf16>(row, slot_bytes<T>(k, 9), col, static_cast<__bf16>(rho));
    }
    static __device__ __forceinline__ void store_init(T* row, const StepConst& k, int a, unsigned col, double v,
                                                      double rho, double rho_dest) {
        const double w = a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        const double sd = (double)round_scale((float)rho_dest);
        at(row + a * k.pitch, col) = static_cast<T>(static_cast<float>(v / sd - w));
        if (a == 0) at(reinterpret_cast<__bf16*>(row + 9 * k.pitch), col) = static_cast<__bf16>((float)rho);
    }
};

template <> struct Codec<kStoreF16> : CodecGlobal<_Float16> {};
template <> struct Codec<kStoreBF16> : CodecGlobal<__bf16> {};
template <> struct Codec<kStoreF16Local> : CodecLocal<_Float16> {};
template <> struct Codec<kStoreBF16Local> : CodecLocal<__bf16> {};
template <> struct Codec<kStoreF16Dest> : CodecDest {};

// ---------------------------------------------------------------- streaming (Eq. 5)
// Velocity ordering: 0 rest; 1 (1,0); 2 (0,1); 3 (-1,0); 4 (0,-1);
// 5 (1,1); 6 (-1,1); 7 (-1,-1); 8 (1,-1).  Opposites 1-3, 2-4, 5-7, 6-8.
//
// Pull: f_a(x, y, t) = f*_a(x - e_a, t - 1).  At a wall (halfway bounce-back)
// the population that would come from outside is the reversed one that left
// the same site: f_a(x, t) = f*_abar(x, t - 1).
// Row addresses are wave-uniform (scalar registers); each lane adds only its
// 32-bit column offset, so every access is a scalar base plus a vector offset.
// xm, xc, xp are byte offsets of columns x-1, x, x+1 within a row.
template <int S, bool WALLS>
__device__ __forceinline__ void pull_row(const typename Codec<S>::T* __restrict__ fin,
                                         const StepConst& k, int y, unsigned xm, unsigned xc,
                                         unsigned xp, float f[9])
{
    using C = Codec<S>;
    using T = typename C::T;
    int ya = y - 1, yb = y + 1;
    bool bot = false, top = false;
    if (WALLS) {
        bot = ya < 0;
        top = yb >= k.ny;
    } else {
        if (ya < 0) ya += k.ny;
        if (yb >= k.ny) yb -= k.ny;
    }
    // At a wall the three populations of a row group come from the reversed
    // populations of the same site: select population, row and column (wave-uniform
    // choices; opposite directions have equal lattice weights and offsets).
    const T* r0 = fin + (long long)y * k.row_stride;
    const T* ra = fin + (long long)(bot ? y : ya) * k.row_stride;
    const T* rb = fin + (long long)(top ? y : yb) * k.row_stride;
    const unsigned x5 = bot ? xc : xm, x6 = bot ? xc : xp;
    const unsigned x7 = top ? xc : xp, x8 = top ? xc : xm;
    f[0] = C::load(r0, k, 0, xc);
    f[1] = C::load(r0, k, 1, xm);
    f[3] = C::load(r0, k, 3, xp);
    f[2] = C::load(ra, k, bot ? 4 : 2, xc);
    f[5] = C::load(ra, k, bot ? 7 : 5, x5);
    f[6] = C::load(ra, k, bot ? 8 : 6, x6);
    f[4] = C::load(rb, k, top ? 2 : 4, xc);
    f[7] = C::load(rb, k, top ? 5 : 7, x7);
    f[8] = C::load(rb, k, top ? 6 : 8, x8);
    if constexpr (C::kDestScaled) {
        const float sc = C::scale(r0, k, xc);
        const float sw0 = sc * (4.0f / 9.0f), sw1 = sc * (1.0f / 9.0f), sw2 = sc * (1.0f / 36.0f);
        f[0] = fmaf(f[0], sc, sw0);
#pragma unroll
        for (int a = 1; a < 5; ++a) f[a] = fmaf(f[a], sc, sw1);
#pragma unroll
        for (int a = 5; a < 9; ++a) f[a] = fmaf(f[a], sc, sw2);
    }
}

__device__ __forceinline__ float density(const float f[9])
{
    // Eq. (6): rho = sum_a f_a  (rest + axis + diagonal partial sums)
    return f[0] + ((f[1] + f[3]) + (f[2] + f[4])) + ((f[5] + f[7]) + (f[6] + f[8]));
}

// Eq. (30) in FP64 for the diagnostics reductions (the liquid pressure is a
// small difference of two large terms).
__device__ __forceinline__ double p_eos_f64(double rho, double b4, double RT, double a)
{
    const double eta = b4 * rho;
    const double om = 1.0 - eta;
    const double num = 1.0 + eta * (1.0 + eta * (1.0 - eta));
    return rho * (RT * num / (om * om * om) - a * rho);
}

// Eq. (23) in FP64: exp(-1/rho) for epsilon = 0, (rho / (epsilon + rho))^(1/epsilon)
// otherwise (rho > 0).
__device__ __forceinline__ double psi_ss_f64(double rho, double eps)
{
    return eps == 0.0 ? exp(-1.0 / rho) : pow(rho / (eps + rho), 1.0 / eps);
}

// psi^2 in FP64 (0 where psi is undefined: rho <= 0, or psi^2 <= 0 for Eq. (24)).
__device__ __forceinline__ double psi2_f64(double rho, const PsiConst& c)
{
    if (c.form == kPsiSS) {
        if (!(rho > 0.0)) return 0.0;
        const double s = psi_ss_f64(rho, c.eps);
        return s * s;
    }
    const double s2 = 2.0 * (p_eos_f64(rho, c.b4, c.RT, c.a) - rho / 3.0) / c.G;
    return s2 > 0.0 ? s2 : 0.0;
}

// Bulk pressure in FP64: rho c_s^2 + G psi^2 / 2, the bulk terms of the pressure
// tensor of Eqs. (18)-(21); with the Eq. (24) psi this is p_EOS of Eq. (30).
__device__ __forceinline__ double pressure_f64(double rho, const PsiConst& c)
{
    if (c.form == kPsiSS) return rho / 3.0 + 0.5 * c.G * psi2_f64(rho, c);
    return p_eos_f64(rho, c.b4, c.RT, c.a);
}

// Hardware reciprocal refined by one Newton step.
__device__ __forceinline__ float recip(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}
// x * rsq(x) refined by one Newton step on the square root.
__device__ __forceinline__ float root(float x)
{
    const float y = __builtin_amdgcn_rsqf(x);
    const float s = x * y;
    return fmaf(fmaf(-s, s, x), 0.5f * y, s);
}

// Eq. (30) Carnahan-Starling pressure.
__device__ __forceinline__ float p_eos(float rho, const StepConst& k)
{
    const float eta = k.b4 * rho;
    const float om = 1.0f - eta;
    const float num = fmaf(eta, fmaf(eta, 1.0f - eta, 1.0f), 1.0f);  // 1 + eta + eta^2 - eta^3
    const float inv = recip(om * om * om);
    return rho * fmaf(k.RT * num, inv, -k.a * rho);
}

// PSI = kPsiCS: Eq. (24), psi = sqrt(2 (p_EOS - rho/3) / G).  Flags non-finite
// rho, b rho/4 >= 1 and psi^2 <= 0; psi is then taken as 0 so the step stays
// finite-cost.  The reciprocals and the square root here and for 1/rho are the
// hardware approximations refined by one Newton step (recip, root), not the raw
// 1-ulp approximations: the force of Eq. (7) takes differences of neighbouring
// psi values, so an ulp-level staircase error in psi becomes force noise, which
// in FP32 roughly quadruples the drift from the FP64 solution over 10^3 steps.
// PSI = kPsiSS: Eq. (23), exp(-1/rho) or (rho / (epsilon + rho))^(1/epsilon);
// flags a non-finite or non-positive rho (psi is then 0).  The form is a template
// parameter so that the Eq. (24) step carries no trace of the other.
template <int PSI = kPsiCS>
__device__ __forceinline__ float pseudopotential(float rho, const StepConst& k, bool& bad)
{
    if constexpr (PSI == kPsiSS) {
        const bool ok = (rho > 0.0f) && (rho < __builtin_huge_valf());
        bad |= !ok;
        if (!ok) return 0.0f;
        return k.psi_eps == 0.0f ? expf(-recip(rho)) : powf(rho * recip(k.psi_eps + rho), k.inv_psi_eps);
    }
    const float psi2 = k.two_over_G * (p_eos(rho, k) - rho * (1.0f / 3.0f));
    const bool ok = (psi2 > 0.0f) && (k.b4 * rho < 1.0f);
    bad |= !ok;
    return ok ? root(psi2) : 0.0f;
}

// Eq. (7) with w(1) = 1/3, w(2) = 1/12, written out per neighbour:
// psi rows m (y-1), c (y), p (y+1); columns L (x-1), C (x), R (x+1).
__device__ __forceinline__ void force_stencil(float mL, float mC, float mR, float cL, float cC,
                                              float cR, float pL, float pC, float pR,
                                              const StepConst& k, float& Fx, float& Fy,
                                              float& Fs2)
{
    const float sx = (1.0f / 3.0f) * (cR - cL) + (1.0f / 12.0f) * ((pR - pL) + (mR - mL));
    const float sy = (1.0f / 3.0f) * (pC - mC) + (1.0f / 12.0f) * ((pR + pL) - (mR + mL));
    const float g = k.negG * cC;
    Fx = g * sx;
    Fy = g * sy;
    // |F|^2 / psi^2 = G^2 |sum w psi e|^2: the improved term of Eq. (25) needs no division
    Fs2 = sx * sx + sy * sy;
}

// Eq. (7) over the 24 sites with |e|^2 in {1, 2, 4, 5, 8} (nearest and next-nearest
// neighbours, Sec. III.B), weights 4/21, 4/45, 1/60, 2/315, 1/5040: the weights whose
// moments are isotropic to eighth order with sum w e_x^2 = 1 (so the bulk term
// G psi^2 / 2 is that of the nearest-neighbour stencil).  P[j][c] is psi at row
// y - 2 + j, column x - 2 + c.  Each weight multiplies differences psi(x + e) -
// psi(x - e) whose +e_y / -e_y partners are added as a pair, and sx, sy are formed
// in the same order with the roles of x and y swapped, so that mirrored or
// transposed neighbourhoods give mirrored or swapped (sx, sy) exactly.
__device__ __forceinline__ void force_stencil_mr(const float (&P)[5][5], const StepConst& k, float& Fx,
                                                 float& Fy, float& Fs2)
{
    constexpr float w1 = 4.0f / 21.0f, w2 = 4.0f / 45.0f, w4 = 1.0f / 60.0f, w5 = 2.0f / 315.0f,
                    w8 = 1.0f / 5040.0f;
    // (u, v) = (1, 0), (1, 1), (1, 2), (2, 0), (2, 1), (2, 2): |e|^2 = 1, 2, 5, 4, 5, 8
    const float dx10 = P[2][3] - P[2][1];
    const float dy10 = P[3][2] - P[1][2];
    const float dx11 = (P[3][3] - P[3][1]) + (P[1][3] - P[1][1]);
    const float dy11 = (P[3][3] - P[1][3]) + (P[3][1] - P[1][1]);
    const float dx12 = (P[4][3] - P[4][1]) + (P[0][3] - P[0][1]);
    const float dy12 = (P[3][4] - P[1][4]) + (P[3][0] - P[1][0]);
    const float dx20 = P[2][4] - P[2][0];
    const float dy20 = P[4][2] - P[0][2];
    const float dx21 = (P[3][4] - P[3][0]) + (P[1][4] - P[1][0]);
    const float dy21 = (P[4][3] - P[0][3]) + (P[4][1] - P[0][1]);
    const float dx22 = (P[4][4] - P[4][0]) + (P[0][4] - P[0][0]);
    const float dy22 = (P[4][4] - P[0][4]) + (P[4][0] - P[0][0]);
    // sum_e w(|e|^2) e_x psi(x + e): weight times |e_x| = u for each pair group
    float sx = w1 * dx10;
    sx = fmaf(w2, dx11, sx);
    sx = fmaf(w5, dx12, sx);
    sx = fmaf(2.0f * w4, dx20, sx);
    sx = fmaf(2.0f * w5, dx21, sx);
    sx = fmaf(2.0f * w8, dx22, sx);
    float sy = w1 * dy10;
    sy = fmaf(w2, dy11, sy);
    sy = fmaf(w5, dy12, sy);
    sy = fmaf(2.0f * w4, dy20, sy);
    sy = fmaf(2.0f * w5, dy21, sy);
    sy = fmaf(2.0f * w8, dy22, sy);
    const float g = k.negG * P[2][2];
    Fx = g * sx;
    Fy = g * sy;
    Fs2 = sx * sx + sy * sy;  // |F|^2 / psi^2 / G^2, as for the nearest-neighbour stencil
}

// MRT collision of Eq. (4) with the forcing of Eq. (25), applied as
// f* = f + M^-1 (m* - m) with M the orthogonal D2Q9 basis (rows rho, e, eps,
// jx, qx, jy, qy, pxx, pxy; norms 9, 36, 36, 6, 12, 6, 12, 4, 4).
// With v from Eq. (6): m*_rho - m_rho = 0 and m*_j - m_j = F exactly.
// (1 - s/2) times the extra Eq. (25) terms equals +12 sigma G^2 s_e |Fs|^2 for e
// and -12 sigma G^2 s_zeta |Fs|^2 for eps.
// Every expression is written so that mirroring the site in x or in y (which
// negates vx, Fx, m_qx, m_xy or their y counterparts) negates or keeps each
// intermediate exactly: a mirror-symmetric state stays mirror-symmetric.
__device__ __forceinline__ void collide(float f[9], float rho, float vx, float vy, float Fx,
                                        float Fy, float Fs2, const StepConst& k)
{
    const float s13 = f[1] + f[3], s24 = f[2] + f[4];
    const float s57 = f[5] + f[7], s68 = f[6] + f[8];
    const float ax = s13 + s24;
    const float dg = s57 + s68;
    const float m_e = fmaf(-4.0f, f[0], fmaf(2.0f, dg, -ax));
    const float m_z = fmaf(4.0f, f[0], fmaf(-2.0f, ax, dg));
    const float d57 = f[5] - f[7], d68 = f[6] - f[8];
    const float m_qx = fmaf(-2.0f, f[1] - f[3], d57 - d68);
    const float m_qy = fmaf(-2.0f, f[2] - f[4], d57 + d68);
    const float m_xx = s13 - s24;
    const float m_xy = s57 - s68;

    const float vF = vx * Fx + vy * Fy;
    const float v2 = vx * vx + vy * vy;
    const bool liq = rho >= k.rho_switch;
    const float a_nu = liq ? k.a_nu_l : k.a_nu_g;
    const float b_nu = liq ? k.b_nu_l : k.b_nu_g;

    // (m* - m) / norm for the non-conserved moments (Eq. 4, Eq. 3, Eq. 25)
    const float te = fmaf(-k.a_e, fmaf(-rho, fmaf(3.0f, v2, -2.0f), m_e), fmaf(k.b_e, vF, k.c_e * Fs2));
    const float tz = fmaf(-k.a_z, fmaf(-rho, fmaf(-3.0f, v2, 1.0f), m_z), -fmaf(k.b_z, vF, k.c_z * Fs2));
    const float qx = fmaf(-k.a_q, fmaf(rho, vx, m_qx), -k.b_q * Fx);
    const float qy = fmaf(-k.a_q, fmaf(rho, vy, m_qy), -k.b_q * Fy);
    const float pxx = fmaf(-a_nu, fmaf(-rho, vx * vx - vy * vy, m_xx), b_nu * (vx * Fx - vy * Fy));
    const float pxy = fmaf(-a_nu, fmaf(-rho, vx * vy, m_xy), (0.5f * b_nu) * (vx * Fy + vy * Fx));

    // f* = f + M^-1 dm  (column k of M^-1 is row k of M divided by its norm)
    const float jx = Fx * (1.0f / 6.0f), jy = Fy * (1.0f / 6.0f);
    const float c_ax = fmaf(-2.0f, tz, -te);
    const float c_dg = fmaf(2.0f, te, tz);
    f[0] += 4.0f * (tz - te);
    const float ux = fmaf(-2.0f, qx, jx), uy = fmaf(-2.0f, qy, jy);
    const float t13 = c_ax + pxx, t24 = c_ax - pxx;
    f[1] += t13 + ux;
    f[3] += t13 - ux;
    f[2] += t24 + uy;
    f[4] += t24 - uy;
    const float xp = jx + qx, yp = jy + qy;
    const float d57p = c_dg + pxy, d68p = c_dg - pxy;
    f[5] += (d57p + xp) + yp;
    f[6] += (d68p - xp) + yp;
    f[7] += (d57p - xp) - yp;
    f[8] += (d68p + xp) - yp;
}

// Workgroups are dispatched round-robin over the XCDs (block b runs on XCD
// b mod 8).  Renumber them so that each XCD receives one contiguous run of
// tiles: neighbouring strips (which share halo rows, halo columns and partly
// written cache lines at tile edges) then mostly meet in the same L2.  The map
// is a permutation of block ids, so results do not depend on it.
__device__ __forceinline__ int logical_block(int b, int nb)
{
    const int per = nb / kNumXcd, rem = nb % kNumXcd;
    const int xcd = b % kNumXcd, idx = b / kNumXcd;
    return (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + idx;
}

__device__ __forceinline__ float lane_from_left(float v) { return __shfl_up(v, 1, kWave); }
__device__ __forceinline__ float lane_from_right(float v) { return __shfl_down(v, 1, kWave); }

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

}  // namespace lbmp
